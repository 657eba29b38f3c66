// HIP kernels of libsq for gfx950 (MI355X): spectral-quadrature density step of
// SQDFT (arXiv 1708.07913, Sec. 3.2-3.3).
//
// Recurrence kernels (Lanczos bounds and Chebyshev moments) -- one workgroup
// per region of influence at a time, persistent over nodes:
//   * a thread owns one, two or three y-adjacent z-columns of the cube (by
//     cube side; see Shape); the current vector t^k of those columns lives in
//     VGPRs (z-neighbours of the stencil come from registers);
//   * x/y neighbours come from a zero-padded LDS plane of t^k that is rewritten
//     once per z (double-buffered, one barrier per plane, or two planes per
//     barrier in the kernels built with PPB = 2); the zero halo is the
//     Dirichlet truncation of Sec. 3.1;
//   * t^{k-1} streams through a per-workgroup global slot that is read and
//     overwritten with t^k in the same sweep (two vector passes per step);
//   * the nonlocal projectors of every atom image in the region are applied
//     inside the sweep through per-column z-runs built once per node; their
//     dot products with the new vector are accumulated along each run and
//     added into LDS at the run's end;
//   * workgroups walk node ranges split by XCD (blockIdx % 8) so that one
//     XCD's L2 holds neighbouring V_eff windows and projector tables.
// FP32-mixed: vectors, LDS plane and potential window stored in FP32; every
// operand is widened to FP64 before it is used, so the arithmetic (stencil
// sum, projector terms, update, dots) is FP64 and the one rounding per step
// is the FP32 store of t^{k+1}.
#include <hip/hip_runtime.h>

#include "sq_internal.h"

#include <math.h>

#include <mutex>
#include <type_traits>

namespace sq {
#if SQ_TWO_ROWS
namespace two_rows {
#endif
namespace {

constexpr int NO = kNoMax;

// Prefetch depths (planes) of the vectors the ring kernels read from their
// workgroup slots: t^{k-1} in the moments sweep, x_{j-1} and x_{j-2} in the
// Lanczos formation.
#ifndef SQ_MOMENTS_AHEAD
#define SQ_MOMENTS_AHEAD 1
#endif
#ifndef SQ_LANCZOS_AHEAD
#define SQ_LANCZOS_AHEAD 1
#endif
// Two-row build of the 21-27-point cubes (a second object of this file; its
// kernels live in namespace sq::two_rows, opened above when the build defines
// SQ_TWO_ROWS=1; left undefined, the preprocessor reads it as 0 there)
#ifndef SQ_TWO_ROWS
#define SQ_TWO_ROWS 0
#endif
constexpr int kMomentsAhead = SQ_MOMENTS_AHEAD;
// FP32-mixed moments: leading steps run in FP64 (see moments_mixed_kernel)
constexpr int kMixedFp64Steps = 4;
constexpr int kLanczosAhead = SQ_LANCZOS_AHEAD;

// Smallest row stride >= pe for which a step from (x = xw - 1, y) to
// (x = 0, y + rb) moves the address by 1 modulo 32 (see Shape::P); the cube
// side c is not needed beyond xw and pe.
constexpr int plane_stride(int c, int rb, int xw, int pe) {
    if (xw == 32) return pe;
    for (int p = pe; p < pe + 32; ++p)
        if (((rb * p - xw) % 32 + 32) % 32 == 0) return p;
    return pe;  // no such stride (even rb with odd xw): keep the plain layout
}

template <int C>
struct Shape {
    static constexpr int RB = rows_per_thread(C, SQ_TWO_ROWS);
    static constexpr int CC = C * C;
    static constexpr int YP = (C + RB - 1) / RB;            // row groups
    // 29- and 31-point cubes give each row group 32 lanes (the last idle or
    // two): a half-wave then reads 32 consecutive plane entries, which keeps
    // the 64-bit LDS reads free of bank conflicts
    static constexpr int XW = row_group_threads(C, SQ_TWO_ROWS);  // threads per row group
    static constexpr int NT = XW * YP;                       // threads owning row groups
    static constexpr int SP = (int)slot_plane(C, SQ_TWO_ROWS);  // doubles per slot plane
    static constexpr int PE = C + 2 * NO;                    // padded plane edge (zero halo NO)
    // Row stride of the plane.  With XW = C the lanes of a wave run along x
    // and step to the next row group at x = C; a stride with
    // RB * P = XW (mod 32) makes that step advance the 8-byte address by one,
    // so any 32 consecutive lanes touch 32 distinct bank pairs for every
    // uniform (dx, dy) offset.  The 32-lane row groups need no padding.
    static constexpr int P = plane_stride(C, RB, XW, PE);
    // + RB + 1 rows read (and discarded) by columns past the cube edge
    static constexpr int ROWS = PE + RB + 1;
    static constexpr int PLANE = ROWS * P + 1;               // + one write-only cell for idle threads
    static constexpr int IDLE_CORNER = 0;                    // idle threads read real cells and discard them
    static constexpr int IDLE_WRITE = ROWS * P;
    static constexpr int BLOCK = (NT + 63) / 64 * 64;
    static constexpr int NW = BLOCK / 64;
    static constexpr int MAXRUNS = (C > kResidentCube ? 4 : 6) * CC + 512;
    // whole columns of the current vector stay in registers up to kResidentCube;
    // wider regions stream it through the workgroup's buffers with a window of
    // 2 NO + 2 planes in registers
    static constexpr bool STREAM = C > kResidentCube;
    // plane buffers: two for the streamed kernels (one plane per barrier);
    // four for the register-ring kernels, which use two, or all four with
    // two planes per barrier
    static constexpr int NBUF = STREAM ? 2 : 4;
    static constexpr int CPT = (CC + BLOCK - 1) / BLOCK;     // columns per thread in the set-up scan
};

// Run record: x = image slot | z_first << 8 | z_last << 16 | chain << 24,
// y = value base (value at plane z is pvals[y + z]).  The sentinel never
// becomes active and never ends.
constexpr unsigned kSentinelX = (0xFEu << 16) | (0xFFu << 8);
constexpr unsigned kIdleOffset = 0x7FFFFF00u;  // beyond every buffer: loads read 0, stores drop

template <int C, typename T, int NCH>
struct Lds {
    T plane[Shape<C>::NBUF][Shape<C>::PLANE];  // double-buffered groups of planes
    uint2 runs[Shape<C>::MAXRUNS + 1];
    int col_start[Shape<C>::CC + 1];
    int col_fill[Shape<C>::CC];
    int col_off[Shape<C>::CC][NCH];  // first record of each chain, relative to col_start
    int img_atom[kMaxImages];
    int img_lb[kMaxImages][3];
    int img_prefix[kMaxImages + 1];
    int img_run0[kMaxImages];
    int img_nrun[kMaxImages];
    double img_coef[kMaxImages];
    double s[2][kMaxImages];
    double cs[kMaxImages];
    double red[Shape<C>::NW * 4];
    double bc[4];
    int scan_tot[Shape<C>::NW];
    int ni;
    int bad;
    int nch;  // chains needed by this region (max sphere overlap depth, >= 1)
    int ps;   // plane stride of the projector value boxes (doubles)
    int item; // work-queue index taken by the workgroup
};

struct LanczosLds {
    double al[kMaxLanczos];
    double be[kMaxLanczos];
};

__device__ __forceinline__ int floor_div(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__device__ __forceinline__ int ceil_div(int a, int b) { return -floor_div(-a, b); }
__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Raw buffer access: SGPR descriptor + one VGPR byte offset + SGPR byte offset,
// so that per-plane addresses stay scalar.  Out-of-range offsets read 0 and
// drop stores (used for idle columns).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// A thread's RB rows at one plane of a thread-interleaved slot (Lanczos ring
// kernel): one 8- or 16-byte access per thread, so a wave moves one
// contiguous, line-aligned block.  The moments ring kernel keeps one access
// per row: with the paired access it spilled more and ran 21 % slower.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int RB>
__device__ __forceinline__ void slot_load(double (&v)[RB], __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    static_assert(RB == 1 || RB == 2, "one or two rows per thread");
    if constexpr (RB == 1) {
        v[0] = bload<double>(r, voff, soff);
    } else {
        const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        v[0] = __builtin_bit_cast(double, u32x2{q.x, q.y});
        v[1] = __builtin_bit_cast(double, u32x2{q.z, q.w});
    }
}
template <int RB>
__device__ __forceinline__ void slot_store(const double (&v)[RB], __amdgpu_buffer_rsrc_t r, unsigned voff,
                                           unsigned soff) {
    static_assert(RB == 1 || RB == 2, "one or two rows per thread");
    if constexpr (RB == 1) {
        bstore(v[0], r, voff, soff);
    } else {
        const u32x2 a = __builtin_bit_cast(u32x2, v[0]), b = __builtin_bit_cast(u32x2, v[1]);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{a.x, a.y, b.x, b.y}, r, voff, soff, 0);
    }
}

// Keep a running sum materialised where it is updated.  Without this the
// compiler sinks a chain of per-plane accumulations to its single use after
// the unrolled sweep and keeps every operand live until then.  Emits nothing.
__device__ __forceinline__ void pin(double &x) { asm volatile("" : "+v"(x)); }

// A workgroup-uniform double, moved to SGPRs (VALU ops then take it as their
// scalar operand instead of holding a copy per lane).
__device__ __forceinline__ double uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// The thread index as a value the compiler cannot relate to earlier uses:
// addresses derived from it are formed where they are needed instead of being
// kept live (and spilled) through the unrolled sweeps.
__device__ __forceinline__ int fresh_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Butterfly sum over the 64 lanes.  The lane index is made opaque so that the
// permute addresses are formed here rather than hoisted and kept live (they
// would otherwise occupy registers through the whole sweep).
__device__ __forceinline__ double wave_sum(double v) {
    int lane = (int)__lane_id();
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int src = (lane ^ off) << 2;
        const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
        const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
        v += __hiloint2double(hi, lo);
    }
    return v;
}

// Sum of (a, b) over the workgroup; the result is returned to every thread.
template <int C, typename T, int NCH>
__device__ __forceinline__ void block_sum2(Lds<C, T, NCH> &L, double &a, double &b, int tid) {
    constexpr int NW = Shape<C>::NW;
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
        L.red[2 * w] = a;
        L.red[2 * w + 1] = b;
    }
    __syncthreads();
    if (tid < 2) {
        double s = 0.0;
        for (int i = 0; i < NW; ++i) s += L.red[2 * i + tid];
        L.bc[tid] = s;
    }
    __syncthreads();
    a = uniform(L.bc[0]);
    b = uniform(L.bc[1]);
    __syncthreads();
}

// SplitMix64 (S. Vigna): first output for a given seed, mapped to [0, 1).
__device__ __forceinline__ double unit_from_seed(unsigned long long seed) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ unsigned run_key(uint2 r, bool with_chain) {
    // (chain, z_first, image slot)
    return (with_chain ? (((r.x >> 24) & 3u) << 16) : 0u) | (((r.x >> 8) & 0xFFu) << 8) | (r.x & 0xFFu);
}

__device__ void sort_runs(uint2 *runs, int b, int e, bool with_chain) {
    for (int i = b + 1; i < e; ++i) {
        const uint2 r = runs[i];
        const unsigned key = run_key(r, with_chain);
        int j = i - 1;
        while (j >= b && run_key(runs[j], with_chain) > key) {
            runs[j + 1] = runs[j];
            --j;
        }
        runs[j + 1] = r;
    }
}

// ---------------------------------------------------------------------------
// Region of influence of node q: projector images meeting the cube and, per
// cube column, the clipped z-runs of their spheres split into chains of
// disjoint runs (more than one chain only where spheres overlap).
// ---------------------------------------------------------------------------
template <int C, typename T, int NCH, typename AT>
__device__ void setup_region(const AT &A, Lds<C, T, NCH> &L, int qi, int qj, int qk, int tid) {
    using S = Shape<C>;
    const int n = A.n, m = A.m;
    if (tid == 0) {
        L.ni = 0;
        L.bad = 0;
        L.nch = 1;
        L.ps = A.pstride;
        L.runs[S::MAXRUNS] = make_uint2(kSentinelX, 0u);
    }
    for (int i = tid; i < S::NBUF * S::PLANE; i += S::BLOCK) (&L.plane[0][0])[i] = T(0);
    for (int i = tid; i < S::CC; i += S::BLOCK) L.col_fill[i] = 0;
    for (int i = tid; i < kMaxImages; i += S::BLOCK) L.s[0][i] = L.s[1][i] = 0.0;
    __syncthreads();

    // every lattice image (atom a, translation t) whose sphere's box meets the cube
    const int lo0 = qi - m, lo1 = qj - m, lo2 = qk - m;
    for (int a = tid; a < A.natom; a += S::BLOCK) {
        const AtomDev at = A.atoms[a];
        const int tl0 = ceil_div(lo0 - at.bx - at.dmax[0], n), th0 = floor_div(lo0 + C - 1 - at.bx - at.dmin[0], n);
        const int tl1 = ceil_div(lo1 - at.by - at.dmax[1], n), th1 = floor_div(lo1 + C - 1 - at.by - at.dmin[1], n);
        const int tl2 = ceil_div(lo2 - at.bz - at.dmax[2], n), th2 = floor_div(lo2 + C - 1 - at.bz - at.dmin[2], n);
        for (int tz = tl2; tz <= th2; ++tz)
            for (int ty = tl1; ty <= th1; ++ty)
                for (int tx = tl0; tx <= th0; ++tx) {
                    const int slot = atomicAdd(&L.ni, 1);
                    if (slot < kMaxImages) {
                        L.img_atom[slot] = a;
                        L.img_lb[slot][0] = at.bx + n * tx - lo0;
                        L.img_lb[slot][1] = at.by + n * ty - lo1;
                        L.img_lb[slot][2] = at.bz + n * tz - lo2;
                        L.img_coef[slot] = at.coef;
                        L.img_run0[slot] = at.run0;
                        L.img_nrun[slot] = at.nrun;
                    }
                }
    }
    __syncthreads();
    int ni = L.ni;
    if (ni > kMaxImages) {
        if (tid == 0) atomicOr(A.flags, kFlagImages);
        ni = kMaxImages;
    }
    if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < ni; ++i) {
            L.img_prefix[i] = acc;
            acc += L.img_nrun[i];
        }
        L.img_prefix[ni] = acc;
    }
    __syncthreads();
    const int npairs = L.img_prefix[ni];

    // count, then place, the clipped z-runs of every image column inside the cube
    for (int pass = 0; pass < 2; ++pass) {
        for (int p = tid; p < npairs; p += S::BLOCK) {
            int lo = 0, hi = ni;  // largest I with prefix[I] <= p
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (L.img_prefix[mid] <= p) lo = mid;
                else hi = mid;
            }
            const int I = lo;
            const RunDev r = A.runs[L.img_run0[I] + (p - L.img_prefix[I])];
            const int cx = L.img_lb[I][0] + r.dx, cy = L.img_lb[I][1] + r.dy;
            if (cx < 0 || cx >= C || cy < 0 || cy >= C) continue;
            const int z0 = L.img_lb[I][2] + r.dz0, z1 = z0 + r.len - 1;
            const int zl = z0 > 0 ? z0 : 0, zh = z1 < C - 1 ? z1 : C - 1;
            if (zl > zh) continue;
            const int col = cy * C + cx;
            const int pos = atomicAdd(&L.col_fill[col], 1);
            if (pass == 1 && pos < S::MAXRUNS) {
                L.runs[pos] = make_uint2((unsigned)I | ((unsigned)zl << 8) | ((unsigned)zh << 16),
                                         (unsigned)(r.vstart - z0 * A.pstride));
            }
        }
        __syncthreads();
        if (pass == 0) {
            // exclusive scan of the per-column counts: each thread sums a chunk
            // of CPT columns, then a wave/workgroup scan of the chunk sums
            const int c0 = tid * S::CPT;
            int chunk = 0;
#pragma unroll
            for (int i = 0; i < S::CPT; ++i)
                if (c0 + i < S::CC) chunk += L.col_fill[c0 + i];
            int incl = chunk;
            const int lane = tid & 63;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off, 64);
                if (lane >= off) incl += t;
            }
            if (lane == 63) L.scan_tot[tid >> 6] = incl;
            __syncthreads();
            int base = 0;
            for (int w = 0; w < (tid >> 6); ++w) base += L.scan_tot[w];
            int run = base + incl - chunk;
#pragma unroll
            for (int i = 0; i < S::CPT; ++i) {
                if (c0 + i < S::CC) {
                    const int v = L.col_fill[c0 + i];
                    L.col_start[c0 + i] = run;
                    L.col_fill[c0 + i] = run;
                    run += v;
                }
            }
            if (c0 < S::CC && c0 + S::CPT >= S::CC) {
                L.col_start[S::CC] = run;
                if (run > S::MAXRUNS) L.bad = 1;
            }
            __syncthreads();
        }
    }
    if (L.bad) {
        if (tid == 0) atomicOr(A.flags, kFlagRuns);
        for (int i = tid; i <= S::CC; i += S::BLOCK) L.col_start[i] = 0;
        __syncthreads();
    }
    // per column: sort by z_first, split first-fit into chains of disjoint runs
    // (as many as spheres overlap at one point), chain 0 first
    for (int col = tid; col < S::CC; col += S::BLOCK) {
        const int b = L.col_start[col], e = L.col_start[col + 1];
        sort_runs(L.runs, b, e, false);
        int last[NCH], cnt[NCH];
#pragma unroll
        for (int ci = 0; ci < NCH; ++ci) {
            last[ci] = -1;
            cnt[ci] = 0;
        }
        int used = 1;
        for (int i = b; i < e; ++i) {
            uint2 r = L.runs[i];
            const int zf = (int)((r.x >> 8) & 0xFFu), zl = (int)((r.x >> 16) & 0xFFu);
            int c = -1;
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci)
                if (c < 0 && zf > last[ci]) c = ci;
            if (c < 0) {
                atomicOr(A.flags, kFlagOverlap);
                c = NCH - 1;
            }
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci)
                if (c == ci) {
                    last[ci] = zl;
                    ++cnt[ci];
                }
            if (c + 1 > used) used = c + 1;
            r.x |= (unsigned)c << 24;
            L.runs[i] = r;
        }
        if (used > 1) {
            sort_runs(L.runs, b, e, true);
            atomicMax(&L.nch, used);
        }
        int off = 0;
#pragma unroll
        for (int ci = 0; ci < NCH; ++ci) {
            L.col_off[col][ci] = off;
            off += cnt[ci];
        }
    }
    __syncthreads();
}

// One chain of disjoint z-runs of a column, walked plane by plane without
// branches except at the end of a run.
struct Chain {
    int i, e;       // current record, end of the chain
    unsigned rx;    // slot | z_first << 8 | z_last << 16 of the current record
    int vb;         // value base of the current record (value at plane z: vb + z * ps)
    int ps;         // plane stride of the value boxes (workgroup-uniform)
    double acc;
    double pv;      // projector value at the plane being processed (fetched one plane ahead)

    __device__ __forceinline__ int sl() const { return (int)(rx & 0xFFu); }
    __device__ __forceinline__ int z0() const { return (int)((rx >> 8) & 0xFFu); }
    __device__ __forceinline__ int z1() const { return (int)((rx >> 16) & 0xFFu); }
    __device__ __forceinline__ void load(const uint2 *runs, int sentinel) {
        const uint2 r = runs[i < e ? i : sentinel];
        rx = r.x;
        vb = (int)r.y;
    }
    __device__ __forceinline__ void start(const uint2 *runs, int b, int end, int sentinel, int stride) {
        i = b;
        e = end;
        ps = stride;
        acc = 0.0;
        load(runs, sentinel);
    }
    // issue the load of the projector value at plane z (0 outside the current
    // run); it is consumed one plane later, so its latency overlaps a plane
    __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t pvr, int z) {
        const bool act = (z >= z0()) & (z <= z1());
        pv = bload<double>(pvr, act ? (unsigned)(vb + z * ps) * 8u : kIdleOffset, 0u);
    }
    // after plane z: a finished run adds its dot product into s[slot]
    __device__ __forceinline__ void finish(double *s, int z, const uint2 *runs, int sentinel) {
        if (z == z1()) {
            atomicAdd(&s[sl()], acc);
            acc = 0.0;
            ++i;
            load(runs, sentinel);
        }
    }
};

// The same walk for register-only passes (no barrier to hide latency
// behind): values are fetched two planes ahead, from the current record or
// the next one (after plane z the current record ends at z + 1 or later, so
// plane z + 2 lies in the current record, in the next one, or in neither).
struct Chain2 {
    int i, e;
    unsigned rx, nrx;  // current and next record: slot | z_first << 8 | z_last << 16
    int vb, nvb;       // their value bases
    int ps;            // plane stride of the value boxes (workgroup-uniform)
    double acc;
    double pv[2];      // values of planes z and z + 1 (indexed by plane parity)
    double c;          // per-image coefficient of the current record (second Lanczos pass)

    __device__ __forceinline__ int sl() const { return (int)(rx & 0xFFu); }
    __device__ __forceinline__ int z1() const { return (int)((rx >> 16) & 0xFFu); }
    __device__ __forceinline__ void start(const uint2 *runs, int b, int end, int sentinel, int stride) {
        i = b;
        e = end;
        ps = stride;
        acc = 0.0;
        const uint2 r0 = runs[i < e ? i : sentinel], r1 = runs[i + 1 < e ? i + 1 : sentinel];
        rx = r0.x;
        vb = (int)r0.y;
        nrx = r1.x;
        nvb = (int)r1.y;
    }
    __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t pvr, int z) {
        const bool cur = (z >= (int)((rx >> 8) & 0xFFu)) & (z <= (int)((rx >> 16) & 0xFFu));
        const bool nxt = (z >= (int)((nrx >> 8) & 0xFFu)) & (z <= (int)((nrx >> 16) & 0xFFu));
        const unsigned off =
            cur ? (unsigned)(vb + z * ps) * 8u : (nxt ? (unsigned)(nvb + z * ps) * 8u : kIdleOffset);
        pv[z & 1] = bload<double>(pvr, off, 0u);
    }
    __device__ __forceinline__ void finish(double *s, int z, const uint2 *runs, int sentinel) {
        if (z == z1()) {
            atomicAdd(&s[sl()], acc);
            acc = 0.0;
            ++i;
            rx = nrx;
            vb = nvb;
            const uint2 r1 = runs[i + 1 < e ? i + 1 : sentinel];
            nrx = r1.x;
            nvb = (int)r1.y;
        }
    }
};

// Columns owned by one thread and their per-column addressing.
template <int C>
struct Cols {
    using S = Shape<C>;
    static constexpr int RB = S::RB;
    int x, y0;
    int corner;                 // LDS offset of the thread's neighbourhood corner
    int col[RB];                // cube column index, or -1
    int pcw[RB];                // LDS write offset of the column's plane value
    unsigned slot;              // byte offset of the thread's rows in a slot plane (Lanczos ring)
    __device__ __forceinline__ void init(int tid) {
        const bool t_active = tid < S::NT;
        x = t_active ? tid % S::XW : 0;
        y0 = t_active ? (tid / S::XW) * RB : 0;
        // lanes past the cube's x range read (and discard) the next padded row
        corner = t_active ? y0 * S::P + x : S::IDLE_CORNER;
        slot = (t_active && x < C && y0 < C) ? (unsigned)(((tid / S::XW) * C + x) * RB) * 8u : kIdleOffset;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool ok = t_active && (x < C) && (y0 + r < C);
            col[r] = ok ? (y0 + r) * C + x : -1;
            pcw[r] = ok ? corner + (NO + r) * S::P + NO : S::IDLE_WRITE;
        }
    }
    __device__ __forceinline__ bool valid(int r) const { return col[r] >= 0; }
    // col[r] recomputed from a fresh thread index (see fresh_tid)
    __device__ __forceinline__ static int column(int r) {
        const int t = fresh_tid();
        if (t >= S::NT) return -1;
        const int xx = t % S::XW, yy = (t / S::XW) * RB + r;
        return (xx < C && yy < C) ? yy * C + xx : -1;
    }
};

// Position the chains of a column at their first records and fetch plane 0.
template <int C, typename T, int NCH>
__device__ __forceinline__ void chains_start(const Lds<C, T, NCH> &L, __amdgpu_buffer_rsrc_t pvr, int column,
                                             Chain (&ch)[NCH], int nch) {
    constexpr int SENT = Shape<C>::MAXRUNS;
    const int ps = __builtin_amdgcn_readfirstlane(L.ps);
    const bool ok = column >= 0;
    const int b = ok ? L.col_start[column] : 0;
    const int e = ok ? L.col_start[column + 1] : 0;
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        const int s0 = b + (ok ? L.col_off[column][ci] : 0);
        const int s1 = ci + 1 < NCH ? b + (ok ? L.col_off[column][ci + 1] : 0) : e;
        ch[ci].start(L.runs, s0, s1, SENT, ps);
        ch[ci].pv = 0.0;
        if (ci == 0 || ci < nch) ch[ci].fetch(pvr, 0);
    }
}

template <int C, typename T, int NCH>
__device__ __forceinline__ void chains2_start(const Lds<C, T, NCH> &L, __amdgpu_buffer_rsrc_t pvr, int column,
                                              Chain2 (&ch)[NCH], int nch) {
    constexpr int SENT = Shape<C>::MAXRUNS;
    const int ps = __builtin_amdgcn_readfirstlane(L.ps);
    const bool ok = column >= 0;
    const int b = ok ? L.col_start[column] : 0;
    const int e = ok ? L.col_start[column + 1] : 0;
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        const int s0 = b + (ok ? L.col_off[column][ci] : 0);
        const int s1 = ci + 1 < NCH ? b + (ok ? L.col_off[column][ci + 1] : 0) : e;
        ch[ci].start(L.runs, s0, s1, SENT, ps);
        ch[ci].pv[0] = ch[ci].pv[1] = 0.0;
        if (ci == 0 || ci < nch) {
            ch[ci].fetch(pvr, 0);
            if (C > 1) ch[ci].fetch(pvr, 1);
        }
    }
}

template <int C, int NCH>
__device__ __forceinline__ void chains2_advance(Chain2 (&ch)[NCH], double *s_dst, const uint2 *runs,
                                                __amdgpu_buffer_rsrc_t pvr, int z, int nch) {
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        if (ci == 0 || ci < nch) {
            ch[ci].finish(s_dst, z, runs, Shape<C>::MAXRUNS);
            if (z + 2 < C) ch[ci].fetch(pvr, z + 2);
        }
    }
}

// After plane z of a column: close finished runs into s_dst and fetch plane z + 1.
template <int C, int NCH>
__device__ __forceinline__ void chains_advance(Chain (&ch)[NCH], double *s_dst, const uint2 *runs,
                                               __amdgpu_buffer_rsrc_t pvr, int z, int nch) {
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        if (ci == 0 || ci < nch) {
            ch[ci].finish(s_dst, z, runs, Shape<C>::MAXRUNS);
            if (z + 1 < C) ch[ci].fetch(pvr, z + 1);
        }
    }
}

__device__ __forceinline__ void node_coords(long long q, int n, int &qi, int &qj, int &qk) {
    qi = (int)(q % n);
    qj = (int)((q / n) % n);
    qk = (int)(q / ((long long)n * n));
}

// Projector dots of a vector given plane by plane: s[dst][I] += p_I . t, with
// t(r, z) the value of the thread's column r at plane z.
// AHEAD2 selects the two-plane look-ahead walk (Chain2); the moments kernel
// keeps the one-plane walk, which leaves its register allocation unchanged.
template <bool AHEAD2, int C, typename T, int NCH, typename F>
__device__ __forceinline__ void projector_dots(Lds<C, T, NCH> &L, __amdgpu_buffer_rsrc_t pvr, const Cols<C> &cl,
                                               int dst, int nch, F &&t) {
    constexpr int RB = Shape<C>::RB;
    if constexpr (AHEAD2) {
        Chain2 ch[RB][NCH];
#pragma unroll
        for (int r = 0; r < RB; ++r) chains2_start(L, pvr, Cols<C>::column(r), ch[r], nch);
#pragma unroll
        for (int z = 0; z < C; ++z) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double v = t(r, z);
#pragma unroll
                for (int ci = 0; ci < NCH; ++ci) {
                    if (ci == 0 || ci < nch) {
                        ch[r][ci].acc += ch[r][ci].pv[z & 1] * v;
                        pin(ch[r][ci].acc);
                    }
                }
                chains2_advance<C, NCH>(ch[r], L.s[dst], L.runs, pvr, z, nch);
            }
        }
    } else {
        Chain ch[RB][NCH];
#pragma unroll
        for (int r = 0; r < RB; ++r) chains_start(L, pvr, Cols<C>::column(r), ch[r], nch);
#pragma unroll
        for (int z = 0; z < C; ++z) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double v = t(r, z);
#pragma unroll
                for (int ci = 0; ci < NCH; ++ci) {
                    if (ci == 0 || ci < nch) {
                        ch[r][ci].acc += ch[r][ci].pv * v;
                        pin(ch[r][ci].acc);
                    }
                }
                chains_advance<C, NCH>(ch[r], L.s[dst], L.runs, pvr, z, nch);
            }
        }
    }
    __syncthreads();
}

// The LDS plane of one z, seen from a thread's neighbourhood through three
// base pointers whose stencil offsets all fit the immediate fields of the LDS
// instructions: the NO rows above the thread's rows, the thread's own rows
// (x legs), and the NO rows below.  The plane buffer offset is made opaque per
// plane so that the bases are recomputed (three adds) instead of being kept
// live for every plane of the unrolled sweep.
template <int C, typename T>
struct PlaneView {
    const T *ylo, *xr, *yhi;
    __device__ __forceinline__ PlaneView(const T *plane0, int buf, int corner) {
        constexpr int P = Shape<C>::P, RB = Shape<C>::RB, PLANE = Shape<C>::PLANE;
        int boff = buf * PLANE;
        asm volatile("" : "+s"(boff));
        const T *pl = plane0 + boff + corner;
        ylo = pl + NO;
        xr = pl + NO * P;
        yhi = pl + (NO + RB) * P + NO;
    }
};

// Rows of the y legs for all RB columns of the thread: LDS for the other
// rows, registers for the thread's own rows.
template <int C, typename T>
__device__ __forceinline__ void load_yrows(const PlaneView<C, T> &pv, const T (&tv)[Shape<C>::RB][C], int z,
                                           T (&yrow)[2 * NO + Shape<C>::RB]) {
    constexpr int P = Shape<C>::P, RB = Shape<C>::RB;
#pragma unroll
    for (int j = 0; j < NO; ++j) yrow[j] = pv.ylo[j * P];
#pragma unroll
    for (int r = 0; r < RB; ++r) yrow[NO + r] = tv[r][z];
#pragma unroll
    for (int j = 0; j < NO; ++j) yrow[NO + RB + j] = pv.yhi[j * P];
}

// Stencil part of (H t)[column r, plane z]: sum_d kw[d] (x pair + y pair + z
// pair), x legs from the LDS plane, y legs from `yrow`, z legs from registers.
// A register column value converted where it is used.  For FP32 columns the
// empty asm hides the value from common-subexpression elimination, so the
// compiler does not keep the widened copies of a column live across planes
// (twice the registers of the column itself).
__device__ __forceinline__ double widen_at_use(double v) { return v; }
__device__ __forceinline__ double widen_at_use(float v) {
    asm volatile("" : "+v"(v));
    return (double)v;
}

template <int C, typename T>
__device__ __forceinline__ double stencil_sum(const PlaneView<C, T> &pv, const T (&yrow)[2 * NO + Shape<C>::RB],
                                              const T (&tv)[C], int r, int z, const double (&kw)[NO + 1]) {
    constexpr int P = Shape<C>::P;
    // Every operand is widened before it is added: with FP32 storage the only
    // rounding left in the step is the one of the stored vector.  Two
    // interleaved accumulators (odd and even d) halve the dependent FMA chain.
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int d = 1; d <= NO; ++d) {
        const double xs = (double)pv.xr[r * P + NO + d] + (double)pv.xr[r * P + NO - d];
        const double ys = (double)yrow[NO + r + d] + (double)yrow[NO + r - d];
        double zs = 0.0;
        if (z + d < C) zs = widen_at_use(tv[z + d]);
        if (z - d >= 0) zs = zs + widen_at_use(tv[z - d]);
        acc[d & 1] += kw[d] * (xs + ys + zs);
    }
    return acc[1] + acc[0];
}

// Snapshot arguments and work items are read through the constant address
// space: their addresses are workgroup-uniform, so the fields load into SGPRs.
typedef __attribute__((address_space(4))) const RecurrenceArgs *SnapPtr;
typedef __attribute__((address_space(4))) const WorkItem *ItemPtr;

// The nodes a workgroup processes: one static share of snaps[0] (every node
// q0, q0 + qs, ... < q1 of one XCD's range), or items taken from the queue
// until it is empty.
struct WorkSource {
    int round = 0;
    template <typename LdsT>
    __device__ __forceinline__ bool next(const LaunchArgs &K, LdsT &L, int tid, SnapPtr &Ap, long long &q0,
                                         long long &q1, long long &qs) {
        if (!K.items) {
            if (round++) return false;
            Ap = (SnapPtr)K.snaps;
            const long long nd = Ap->nd;
            const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, lw = blockIdx.x >> 3;
            q0 = nd * xcd / 8 + lw;
            q1 = nd * (xcd + 1) / 8;
            qs = per;
            return true;
        }
        __syncthreads();
        if (tid == 0) L.item = atomicAdd(K.counter, 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(L.item);
        if (idx >= K.n_items) return false;
        const ItemPtr it = (ItemPtr)K.items + idx;
        Ap = (SnapPtr)K.snaps + it->snap;
        q0 = it->q0;
        q1 = it->q1;
        qs = 1;
        return true;
    }
};

// ---------------------------------------------------------------------------
// Chebyshev recurrence and moments (Sec. 3.2):
//   t^0 = e_q, t^1 = Hhat t^0, t^{k+1} = 2 Hhat t^k - t^{k-1},
//   rho^j = t^j[q] (j <= n_pl/2), rho^{2k} = 2 t^k.t^k - rho^0,
//   rho^{2k-1} = 2 t^k.t^{k-1} - rho^1 (k > n_pl/4).
// This kernel serves the cubes wider than kResidentCube (both precisions;
// narrower cubes run the register-ring kernels below): t^k is read from
// buffer X with a look-ahead of NO + 1 planes, t^{k-1} is read from buffer Y
// and replaced there by t^{k+1}; X and Y swap roles every step.  Global loads
// of plane z + 1 (potential window, t^{k-1}, projector values) are issued
// during plane z.
// ---------------------------------------------------------------------------
template <int C, int NCH>
__global__ __launch_bounds__(Shape<C>::BLOCK) void moments_kernel(LaunchArgs K) {
    using S = Shape<C>;
    using T = double;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    constexpr int ZA = NO + 1;  // look-ahead of the streamed t^k
    static_assert(S::STREAM, "streamed cubes only");
    __shared__ Lds<C, T, NCH> L;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    int centre_r = -1;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (cl.col[r] == MC * C + MC) centre_r = r;
    const long long slot_bytes = K.slot_elems * (long long)sizeof(T);
    __amdgpu_buffer_rsrc_t slr =
        make_rsrc(reinterpret_cast<T *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    __amdgpu_buffer_rsrc_t sly =
        make_rsrc(reinterpret_cast<T *>(K.wslots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    unsigned voff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) voff[r] = cl.valid(r) ? (unsigned)cl.col[r] * (unsigned)sizeof(T) : kIdleOffset;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const int npl = A.npl, half = npl / 2;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const double kin0 = -3.0 * A.w[0];

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        const double chi = uniform(A.chi[q]), zeta = uniform(A.zeta[q]);
        const double invz = uniform(1.0 / zeta);
        double kw[NO + 1];
        kw[0] = 0.0;
#pragma unroll
        for (int d = 1; d <= NO; ++d) kw[d] = uniform(-0.5 * A.w[d] * invz);
        const double c0 = uniform(kin0 - chi);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) *
                                        (unsigned)sizeof(T)
                                  : kIdleOffset;
        double *mrow = A.moments + q * (long long)(npl + 1);
        auto e_q = [&](int r, int z) { return T((centre_r == r && z == MC) ? 1 : 0); };

        T tv[RB][C];  // a window of planes of t^k
        if (tid == 0) mrow[0] = 1.0;
        int cur = 0;
        // t^0 goes to X here, so that every sweep reads X
        projector_dots<false>(L, pvr, cl, cur, nch, [&](int r, int z) {
            const T v = e_q(r, z);
            bstore(v, slr, voff[r], (unsigned)(z * S::CC) * (unsigned)sizeof(T));
            return (double)v;
        });

        for (int k = 0; k < half; ++k) {
            const double al = k == 0 ? 1.0 : 2.0;
            const double scale = uniform(al * invz);
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK)
                L.cs[i] = i < ni ? scale * L.img_coef[i] * L.s[cur][i] : 0.0;
            Chain ch[RB][NCH];
#pragma unroll
            for (int r = 0; r < RB; ++r) chains_start(L, pvr, Cols<C>::column(r), ch[r], nch);
            double *snext = L.s[cur ^ 1];
            double d1 = 0.0, d2 = 0.0;
            unsigned zb = (unsigned)__builtin_amdgcn_readfirstlane((int)zbase);
            asm volatile("" : "+s"(zb));  // keep the per-plane offsets inside the step loop
            const bool stream_prev = k > 0;
            // t^k: the first planes of the window
#pragma unroll
            for (int z = 0; z < (ZA < C ? ZA : C); ++z)
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    tv[r][z] = bload<T>(slr, voff[r], (unsigned)(z * S::CC) * (unsigned)sizeof(T));
            // plane 0 loads; plane z + 1 is loaded while plane z is processed
            double vzn[RB], tpn[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                vzn[r] = (double)bload<T>(vr, vcol[r], (unsigned)(n * n) * (zb % (unsigned)n) * (unsigned)sizeof(T));
                tpn[r] = 0.0;
                if (stream_prev) tpn[r] = (double)bload<T>(sly, voff[r], 0u);
            }
#pragma unroll
            for (int z = 0; z < C; ++z) {
                const unsigned sz = (unsigned)(z * S::CC) * (unsigned)sizeof(T);
                double vz[RB], tprev[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    vz[r] = vzn[r];
                    tprev[r] = tpn[r];
                    if (z + 1 < C) {
                        const unsigned sz1 = (unsigned)((z + 1) * S::CC) * (unsigned)sizeof(T);
                        const unsigned vz1 = (unsigned)(n * n) * ((zb + (unsigned)(z + 1)) % (unsigned)n) *
                                             (unsigned)sizeof(T);
                        vzn[r] = (double)bload<T>(vr, vcol[r], vz1);
                        if (stream_prev) tpn[r] = (double)bload<T>(sly, voff[r], sz1);
                    }
                    if (z + ZA < C)
                        tv[r][z + ZA] = bload<T>(slr, voff[r], (unsigned)((z + ZA) * S::CC) * (unsigned)sizeof(T));
                    L.plane[z & 1][cl.pcw[r]] = tv[r][z];
                }
                __syncthreads();
                const PlaneView<C, T> pv(L.plane[0], z & 1, cl.corner);
                T yrow[2 * NO + RB];
                load_yrows<C, T>(pv, tv, z, yrow);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const double acc = stencil_sum<C, T>(pv, yrow, tv[r], r, z, kw);
                    const double tz = (double)tv[r][z];
                    const double u = acc + (vz[r] + c0) * invz * tz;
                    double pval[NCH];
                    double nvd = al * u - tprev[r];
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        pval[ci] = 0.0;
                        if (ci == 0 || ci < nch) {
                            pval[ci] = ch[r][ci].pv;
                            nvd += L.cs[ch[r][ci].sl()] * pval[ci];
                        }
                    }
                    // a column past the cube edge shares its neighbour reads with
                    // a real column; it must stay zero, since it is that column's
                    // y neighbour
                    if (!cl.valid(r)) nvd = 0.0;
                    const double moment = nvd;
                    bstore(nvd, sly, voff[r], sz);  // t^{k+1} over t^{k-1}
                    d1 += nvd * nvd;
                    d2 += nvd * tz;
                    pin(d1);
                    pin(d2);
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        if (ci == 0 || ci < nch) {
                            ch[r][ci].acc += pval[ci] * nvd;
                            pin(ch[r][ci].acc);
                        }
                    }
                    chains_advance<C, NCH>(ch[r], snext, L.runs, pvr, z, nch);
                    if (z == MC && centre_r == r) {
                        mrow[k + 1] = moment;
                        if (k == 0) L.bc[2] = moment;
                        if (fabs(moment) > 1.0 + A.bounds_tol) atomicOr(A.flags, kFlagBounds);
                    }
                }
            }
            __syncthreads();
            // reduce every step: a conditional reduction lets the compiler sink
            // the per-plane products into it and keep them all live
            block_sum2(L, d1, d2, tid);
            if (k + 1 > half / 2) {
                if (tid == 0) {
                    const double r2k = 2.0 * d1 - 1.0, r2k1 = 2.0 * d2 - L.bc[2];
                    mrow[2 * (k + 1)] = r2k;
                    mrow[2 * (k + 1) - 1] = r2k1;
                    if (fabs(r2k) > 1.0 + A.bounds_tol || fabs(r2k1) > 1.0 + A.bounds_tol)
                        atomicOr(A.flags, kFlagBounds);
                }
            }
            // t^k -> t^{k-1}, t^{k+1} -> t^k: X and Y swap
            {
                const __amdgpu_buffer_rsrc_t t = slr;
                slr = sly;
                sly = t;
            }
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) L.s[cur][i] = 0.0;
            cur ^= 1;
            __syncthreads();
        }
    }
    }
}

// ---------------------------------------------------------------------------
// Lanczos spectral bounds (Sec. 3.2): Paige's ordering of the three-term
// recurrence from a fixed SplitMix64 start vector, no reorthogonalisation,
// extreme eigenvalues of the tridiagonal by Sturm counts (a 32-point
// multisection that ends on the bracket bisection reaches).
// ---------------------------------------------------------------------------
__device__ int sturm_count(int k, const double *a, const double *b, double x, double pivmin) {
    int cnt = 0;
    double d = a[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
        d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// Point idx (0..31) of the 32 interior points that split [lo, hi] into 33
// equal parts; the same expression serves the lanes that evaluate the points
// and the lanes that take them over as the new bracket.
__device__ __forceinline__ double split_point(double lo, double hi, int idx) {
    return lo + (hi - lo) * ((double)(idx + 1) / 33.0);
}

// Extreme eigenvalues of the tridiagonal T_k by Sturm counts, on one wave:
// lanes 0-31 bracket the smallest eigenvalue (count target 1), lanes 32-63
// the largest (target k).  A round evaluates the count at 32 interior points
// of the bracket and keeps the sub-interval where it first reaches the
// target, which narrows the bracket 33-fold where bisection halves it.  The
// invariant count(lo) < target <= count(hi) holds throughout; the bracket
// shrinks until no interior point is left (adjacent doubles) and its upper
// end is returned, as with bisection.  out[0] = min, out[1] = max.
__device__ void sturm_extremes(int k, const double *a, const double *b, double *out, int lane) {
    double lo = INFINITY, hi = -INFINITY, bmax2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < k - 1 ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
        if (i < k - 1) bmax2 = fmax(bmax2, b[i] * b[i]);
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(bmax2, 1.0);
    const int half = lane >> 5, j = lane & 31;
    const int target = half ? k : 1;
    for (int round = 0; round < 64; ++round) {
        const double x = split_point(lo, hi, j);
        const bool inside = (x > lo) & (x < hi);
        const unsigned long long in_mask = __builtin_amdgcn_ballot_w64(inside);
        if ((unsigned)(half ? in_mask >> 32 : in_mask) == 0u) break;  // uniform per half
        const bool ge = inside ? sturm_count(k, a, b, x, pivmin) >= target : x >= hi;
        const unsigned long long gm = __builtin_amdgcn_ballot_w64(ge);
        const unsigned g32 = (unsigned)(half ? gm >> 32 : gm);
        const int f = g32 ? __builtin_ctz(g32) : 32;  // first point with count >= target
        const double nlo = f > 0 ? split_point(lo, hi, f - 1) : lo;
        const double nhi = f < 32 ? split_point(lo, hi, f) : hi;
        lo = nlo;
        hi = nhi;
    }
    if (j == 0) out[half] = hi;
}

// Cubes wider than kResidentCube (narrower ones run lanczos_ring_kernel):
// w_j (not yet divided by beta_j) sits in buffer X and v_{j-1} (as the stored
// w_{j-1}) in buffer Y, both read with a look-ahead window and scaled on load.
// The sweep writes the local part u of H v_j - beta_{j-1} v_{j-1} to a third
// buffer; a second pass adds the projector part, forms w = u - alpha v_j over
// Y, and the two buffers swap roles.
template <int C, int NCH>
__global__ __launch_bounds__(Shape<C>::BLOCK) void lanczos_kernel(LaunchArgs K) {
    using S = Shape<C>;
    using T = double;
    constexpr int RB = S::RB;
    constexpr int ZA = NO + 1;
    static_assert(S::STREAM, "streamed cubes only");
    __shared__ Lds<C, T, NCH> L;
    __shared__ LanczosLds LL;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    const long long slot_bytes = K.slot_elems * 8;
    // slr = X (current), sly = Y (previous); wlr: u = H v_j - beta v_{j-1}
    __amdgpu_buffer_rsrc_t slr =
        make_rsrc(reinterpret_cast<T *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    const __amdgpu_buffer_rsrc_t wlr =
        make_rsrc(reinterpret_cast<T *>(K.wslots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    __amdgpu_buffer_rsrc_t sly =
        make_rsrc(reinterpret_cast<T *>(K.xslots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    unsigned voff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) voff[r] = cl.valid(r) ? (unsigned)cl.col[r] * 8u : kIdleOffset;
    const long long ns = (long long)C * C * C;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const double kin0 = -3.0 * A.w[0];
    double kw[NO + 1];
    kw[0] = 0.0;
#pragma unroll
    for (int d = 1; d <= NO; ++d) kw[d] = -0.5 * A.w[d];
    const int kmax = (long long)A.n_lanczos < ns ? A.n_lanczos : (int)ns;
    const double rnorm = 1.0 / A.start_norm;

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) * 8u
                                  : kIdleOffset;
        // v_1[a] = (u(a) - 1/2) / |u - 1/2|, a = local cube index
        auto start = [&](int r, int z) {
            return cl.valid(r) ? (unit_from_seed((unsigned long long)(cl.col[r] + C * C * z)) - 0.5) * rnorm : 0.0;
        };

        double tv[RB][C];  // a window of planes of v_j
        int cur = 0;
        // v_1 goes to X here, so that every sweep reads X
        projector_dots<true>(L, pvr, cl, cur, nch, [&](int r, int z) {
            const double v = start(r, z);
            bstore(v, slr, voff[r], (unsigned)(z * S::CC) * 8u);
            return v;
        });

        double bprev = 0.0, gersh = 0.0;
        // v_j = scx * X, v_{j-1} = scy * Y: the vectors are kept as
        // w = u - alpha v, not divided by beta
        double scx = 1.0, scy = 0.0;
        int ksteps = kmax;
        for (int j = 0; j < kmax; ++j) {
            // Local part of u = H v_j - beta_{j-1} v_{j-1} (stencil and potential)
            // -> wslot.  The projector part, sum_I c_I (p_I . v_j) p_I, is added
            // in the second pass, where the same walk over the projector runs
            // also forms p . w; its contribution to alpha is sum_I c_I (p_I . v_j)^2.
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK)
                L.cs[i] = i < ni ? L.img_coef[i] * L.s[cur][i] : 0.0;
            unsigned zb = (unsigned)__builtin_amdgcn_readfirstlane((int)zbase);
            asm volatile("" : "+s"(zb));
            const __amdgpu_buffer_rsrc_t prev = sly;
            const double sprev = scy;
#pragma unroll
            for (int z = 0; z < (ZA < C ? ZA : C); ++z)
#pragma unroll
                for (int r = 0; r < RB; ++r) tv[r][z] = bload<double>(slr, voff[r], (unsigned)(z * S::CC) * 8u);
            // PPB planes per barrier (one: two plane buffers); the loads of
            // the next plane are issued while this one is processed
            constexpr int PPB = S::NBUF / 2;
            double da = 0.0;
            double vzn[PPB][RB], vpn[PPB][RB];
#pragma unroll
            for (int h = 0; h < PPB; ++h)
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    vzn[h][r] = 0.0;
                    vpn[h][r] = 0.0;
                    if (h < C) {
                        vzn[h][r] = bload<double>(vr, vcol[r], (unsigned)(n * n) * ((zb + (unsigned)h) % (unsigned)n) * 8u);
                        if (j > 0) vpn[h][r] = sprev * bload<double>(prev, voff[r], (unsigned)(h * S::CC) * 8u);
                    }
                }
#pragma unroll
            for (int z0 = 0; z0 < C; z0 += PPB) {
                const int pb = PPB * ((z0 / PPB) & 1);
                double vz[PPB][RB], vprev[PPB][RB];
#pragma unroll
                for (int h = 0; h < PPB; ++h)
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        vz[h][r] = vzn[h][r];
                        vprev[h][r] = vpn[h][r];
                        const int zn = z0 + h + PPB;
                        if (zn < C) {
                            vzn[h][r] = bload<double>(vr, vcol[r], (unsigned)(n * n) * ((zb + (unsigned)zn) % (unsigned)n) * 8u);
                            if (j > 0) vpn[h][r] = sprev * bload<double>(prev, voff[r], (unsigned)(zn * S::CC) * 8u);
                        }
                    }
#pragma unroll
                for (int h = 0; h < PPB; ++h) {
                    const int z = z0 + h;
                    if (z < C) {
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            if (z + ZA < C)
                                tv[r][z + ZA] = bload<double>(slr, voff[r], (unsigned)((z + ZA) * S::CC) * 8u);
                            L.plane[pb + h][cl.pcw[r]] = tv[r][z];
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int h = 0; h < PPB; ++h) {
                    const int z = z0 + h;
                    if (z < C) {
                        const unsigned sz = (unsigned)(z * S::CC) * 8u;
                        const PlaneView<C, double> pv(L.plane[0], pb + h, cl.corner);
                        double yrow[2 * NO + RB];
                        load_yrows<C, double>(pv, tv, z, yrow);
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            double u = scx * (stencil_sum<C, double>(pv, yrow, tv[r], r, z, kw) + (vz[h][r] + kin0) * tv[r][z]);
                            u -= bprev * vprev[h][r];
                            if (!cl.valid(r)) u = 0.0;  // column past the cube edge stays zero
                            bstore(u, wlr, voff[r], sz);
                            da += u * tv[r][z];
                            pin(da);
                        }
                    }
                }
            }
            __syncthreads();
            double dimg = 0.0;
            for (int i = fresh_tid(); i < ni; i += S::BLOCK) dimg += L.cs[i] * L.s[cur][i];
            block_sum2(L, da, dimg, tid);
            const double alpha = uniform(scx * da + dimg);
            double dummy = 0.0;

            // w = u - alpha v_j with the projector part of u added here;
            // beta = |w|;  p . w (taken from w itself: a projector dot carried
            // by linearity, (p.u - alpha p.v) / beta, grows its rounding error by
            // |alpha/beta| per step).  Loads of planes z + 1 and z + 2 are in
            // flight while plane z is processed.
            double db = 0.0;
            Chain2 ch[RB][NCH];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                chains2_start(L, pvr, Cols<C>::column(r), ch[r], nch);
#pragma unroll
                for (int ci = 0; ci < NCH; ++ci) ch[r][ci].c = L.cs[ch[r][ci].sl()];
            }
            // u and v_j loads run LA planes ahead
            constexpr int LA = 3;
            double un[LA][RB], xn[LA][RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
#pragma unroll
                for (int z = 0; z < LA; ++z) {
                    un[z][r] = z < C ? bload<double>(wlr, voff[r], (unsigned)(z * S::CC) * 8u) : 0.0;
                    xn[z][r] = z < C ? bload<double>(slr, voff[r], (unsigned)(z * S::CC) * 8u) : 0.0;
                }
            }
#pragma unroll
            for (int z = 0; z < C; ++z) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    double uz = un[z % LA][r];
                    const double vj = scx * xn[z % LA][r];
                    if (z + LA < C) {
                        const unsigned sz2 = (unsigned)((z + LA) * S::CC) * 8u;
                        un[z % LA][r] = bload<double>(wlr, voff[r], sz2);
                        xn[z % LA][r] = bload<double>(slr, voff[r], sz2);
                    }
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci)
                        if (ci == 0 || ci < nch) uz += ch[r][ci].c * ch[r][ci].pv[z & 1];
                    double w = uz - alpha * vj;
                    if (!cl.valid(r)) w = 0.0;
                    bstore(w, sly, voff[r], (unsigned)(z * S::CC) * 8u);
                    db += w * w;
                    pin(db);
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        if (ci == 0 || ci < nch) {
                            ch[r][ci].acc += ch[r][ci].pv[z & 1] * w;
                            pin(ch[r][ci].acc);
                        }
                    }
                    // a run that ends here hands over to the next record: its
                    // coefficient is read once per run instead of once per plane
                    bool sw[NCH];
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) sw[ci] = z == ch[r][ci].z1();
                    chains2_advance<C, NCH>(ch[r], L.s[cur ^ 1], L.runs, pvr, z, nch);
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci)
                        if ((ci == 0 || ci < nch) && sw[ci]) ch[r][ci].c = L.cs[ch[r][ci].sl()];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            block_sum2(L, db, dummy, tid);
            const double beta = uniform(sqrt(db));
            if (tid == 0) {
                LL.al[j] = alpha;
                LL.be[j] = beta;
                if (!isfinite(alpha) || !isfinite(beta)) atomicOr(A.flags, kFlagLanczos);
            }
            gersh = fmax(gersh, fabs(alpha) + beta + bprev);
            if (j == kmax - 1 || beta <= 1e-13 * gersh) {
                ksteps = j + 1;
                break;
            }
            const double rb = uniform(1.0 / beta);
            {
                // X <- w_j, Y <- the buffer holding v_j
                const __amdgpu_buffer_rsrc_t t = slr;
                slr = sly;
                sly = t;
            }
            scy = scx;
            scx = rb;
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) {
                L.s[cur ^ 1][i] = L.s[cur ^ 1][i] * rb;
                L.s[cur][i] = 0.0;
            }
            cur ^= 1;
            bprev = beta;
            __syncthreads();
        }
        __syncthreads();
        if (tid < 64) sturm_extremes(ksteps, LL.al, LL.be, L.bc, tid);
        __syncthreads();
        if (tid == 0) {
            const double lmn = L.bc[0], lmx = L.bc[1];
            if (A.lmin) A.lmin[q] = lmn;
            if (A.lmax) A.lmax[q] = lmx;
            A.chi[q] = 0.5 * (lmx + lmn);
            A.zeta[q] = (1.0 + A.margin) * 0.5 * (lmx - lmn);
        }
        __syncthreads();
    }
    }
}

// ---------------------------------------------------------------------------
// Register-ring recurrence kernels (cubes whose columns stay in registers).
//
// A thread keeps NR = C + NO + 1 plane slots per owned column.  A sweep reads
// its input vector at ring[z + IN] and writes its output vector at
// ring[z + OUT]: upward sweeps (z = 0 .. C-1) have IN = NO + 1, OUT = 0 and
// downward sweeps the reverse.  The stencil at plane z reaches planes z +- NO,
// so the input plane z - (NO + 1) (upward) held in slot z is dead when the
// output of plane z is written there.  Consecutive steps alternate direction
// and the input of one step is the output of the previous one, so one column
// of slots (instead of one per vector) carries the recurrence.
// ---------------------------------------------------------------------------
template <bool UP> struct RingDir {
    static constexpr int IN = UP ? NO + 1 : 0;
    static constexpr int OUT = UP ? 0 : NO + 1;
    // plane of loop iteration i
    static constexpr __host__ __device__ int plane(int i, int C) { return UP ? i : C - 1 - i; }
};

// One chain of disjoint z-runs walked upward (first record first) or
// downward (last record first).  The sentinel record never becomes active
// and never ends in either direction.
template <bool UP>
struct ChainD {
    int i, b, e;    // current record, chain range [b, e)
    unsigned rx;    // slot | z_first << 8 | z_last << 16
    int vb;         // value base of the current record (value at plane z: vb + z * ps)
    int ps;         // plane stride of the value boxes (workgroup-uniform)
    double acc;
    double pv;      // projector value at the plane being processed

    __device__ __forceinline__ int sl() const { return (int)(rx & 0xFFu); }
    __device__ __forceinline__ int z0() const { return (int)((rx >> 8) & 0xFFu); }
    __device__ __forceinline__ int z1() const { return (int)((rx >> 16) & 0xFFu); }
    __device__ __forceinline__ void load(const uint2 *runs, int sentinel) {
        const bool in = UP ? i < e : i >= b;
        const uint2 r = runs[in ? i : sentinel];
        rx = r.x;
        vb = (int)r.y;
    }
    __device__ __forceinline__ void start(const uint2 *runs, int b0, int e0, int sentinel, int stride) {
        b = b0;
        e = e0;
        ps = stride;
        i = UP ? b0 : e0 - 1;
        acc = 0.0;
        pv = 0.0;
        load(runs, sentinel);
    }
    __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t pvr, int z) {
        const bool act = (z >= z0()) & (z <= z1());
        pv = bload<double>(pvr, act ? (unsigned)(vb + z * ps) * 8u : kIdleOffset, 0u);
    }
    // after plane z: a run that ends here adds its dot product into s[slot]
    __device__ __forceinline__ void finish(double *s, int z, const uint2 *runs, int sentinel) {
        if (z == (UP ? z1() : z0())) {
            atomicAdd(&s[sl()], acc);
            acc = 0.0;
            i += UP ? 1 : -1;
            load(runs, sentinel);
        }
    }
};

template <bool UP, int C, typename T, int NCH>
__device__ __forceinline__ void chainsd_start(const Lds<C, T, NCH> &L, __amdgpu_buffer_rsrc_t pvr, int column,
                                              ChainD<UP> (&ch)[NCH], int nch) {
    constexpr int SENT = Shape<C>::MAXRUNS;
    const int ps = __builtin_amdgcn_readfirstlane(L.ps);
    const bool ok = column >= 0;
    const int b = ok ? L.col_start[column] : 0;
    const int e = ok ? L.col_start[column + 1] : 0;
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        const int s0 = b + (ok ? L.col_off[column][ci] : 0);
        const int s1 = ci + 1 < NCH ? b + (ok ? L.col_off[column][ci + 1] : 0) : e;
        ch[ci].start(L.runs, s0, s1, SENT, ps);
        if (ci == 0 || ci < nch) ch[ci].fetch(pvr, UP ? 0 : C - 1);
    }
}

// After plane z: close finished runs into s_dst and fetch the next plane.
template <bool UP, int C, int NCH>
__device__ __forceinline__ void chainsd_advance(ChainD<UP> (&ch)[NCH], double *s_dst, const uint2 *runs,
                                                __amdgpu_buffer_rsrc_t pvr, int z, int nch) {
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        if (ci == 0 || ci < nch) {
            ch[ci].finish(s_dst, z, runs, Shape<C>::MAXRUNS);
            const int zn = UP ? z + 1 : z - 1;
            if (zn >= 0 && zn < C) ch[ci].fetch(pvr, zn);
        }
    }
}

// Sum of N <= 4 values over the workgroup with a single barrier: every
// thread adds the per-wave sums itself, in the same order (the results are
// identical across threads).  The per-wave slots are not written again
// before the caller's next barrier, so no trailing barrier is needed.
template <int N, int C, typename T, int NCH>
__device__ __forceinline__ void block_sum_once(Lds<C, T, NCH> &L, double (&v)[N], int tid) {
    constexpr int NW = Shape<C>::NW;
    static_assert(N <= 4, "per-wave reduction slots");
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) L.red[N * w + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int ww = 0; ww < NW; ++ww) acc += L.red[N * ww + i];
        v[i] = uniform(acc);
    }
}

// y legs of plane z for all RB columns, own rows from the ring.
template <int C, int IN>
__device__ __forceinline__ void load_yrows_ring(const PlaneView<C, double> &pv,
                                                const double (&R)[Shape<C>::RB][C + NO + 1], int z,
                                                double (&yrow)[2 * NO + Shape<C>::RB]) {
    constexpr int P = Shape<C>::P, RB = Shape<C>::RB;
#pragma unroll
    for (int j = 0; j < NO; ++j) yrow[j] = pv.ylo[j * P];
#pragma unroll
    for (int r = 0; r < RB; ++r) yrow[NO + r] = R[r][z + IN];
#pragma unroll
    for (int j = 0; j < NO; ++j) yrow[NO + RB + j] = pv.yhi[j * P];
}

// Stencil part of (H x)[column r, plane z] with the column's planes in the ring
// at offset IN: sum_d kw[d] (x pair + y pair + z pair).
template <int C, int IN>
__device__ __forceinline__ double stencil_ring(const PlaneView<C, double> &pv, const double (&yrow)[2 * NO + Shape<C>::RB],
                                               const double (&col)[C + NO + 1], int r, int z,
                                               const double (&kw)[NO + 1]) {
    constexpr int P = Shape<C>::P;
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int d = 1; d <= NO; ++d) {
        const double xs = pv.xr[r * P + NO + d] + pv.xr[r * P + NO - d];
        const double ys = yrow[NO + r + d] + yrow[NO + r - d];
        double zs = 0.0;
        if (z + d < C) zs = col[z + d + IN];
        if (z - d >= 0) zs = zs + col[z - d + IN];
        acc[d & 1] += kw[d] * (xs + ys + zs);
    }
    return acc[1] + acc[0];
}

// ---------------------------------------------------------------------------
// FP64 Chebyshev moments on the register ring (Sec. 3.2 recurrence and
// moments).  Per step: t^k in the ring (input layout), t^{k-1} read from the
// workgroup's slot plane by plane and replaced there by t^k, t^{k+1} into the
// ring (output layout): two vector transfers per step.
// ---------------------------------------------------------------------------
struct MomentsStep {
    double al, invz, c0;
    int k;
    bool prev;  // t^{k-1} is read from the slot (k > 0)
    // force mode: u <- ua t^k + u + uc t^{k+1} (ua = c_0 at k = 0, else 0)
    double ua, uc;
};

// FORCE: instead of the moments, accumulate u = sum_j c_j t^j in the vector
// buffer `ur` (same layout as the slot; read and rewritten plane by plane).
template <int C, int NCH, bool UP, int PPB, bool FORCE = false, typename AT>
__device__ __forceinline__ void moments_ring_sweep(const AT &A, Lds<C, double, NCH> &L, const Cols<C> &cl,
                                                   double (&R)[Shape<C>::RB][C + NO + 1],
                                                   __amdgpu_buffer_rsrc_t slr, __amdgpu_buffer_rsrc_t vr,
                                                   __amdgpu_buffer_rsrc_t pvr, const unsigned (&vcol)[Shape<C>::RB],
                                                   const unsigned (&voff)[Shape<C>::RB], unsigned zbase,
                                                   const double (&kw)[NO + 1], const MomentsStep &st,
                                                   double *snext, int nch, int centre_r, double *mrow,
                                                   double &d1, double &d2, __amdgpu_buffer_rsrc_t ur) {
    using S = Shape<C>;
    using D = RingDir<UP>;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    const int n = A.n;
    ChainD<UP> ch[RB][NCH];
#pragma unroll
    for (int r = 0; r < RB; ++r) chainsd_start<UP>(L, pvr, Cols<C>::column(r), ch[r], nch);
    unsigned zb = (unsigned)__builtin_amdgcn_readfirstlane((int)zbase);
    asm volatile("" : "+s"(zb));
    // PPB planes share one barrier (their LDS planes are written together);
    // V_eff runs PPB planes ahead and t^{k-1} TPA planes ahead.  At k = 0 the
    // t^{k-1} loads use the idle offset (they read 0) instead of a branch,
    // which would serialise the prefetch.
    static_assert(PPB == 1 || PPB == 2, "one or two planes per barrier");
    constexpr int TPA = kMomentsAhead > PPB ? kMomentsAhead : PPB;
    unsigned poff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) poff[r] = st.prev ? voff[r] : kIdleOffset;
    double vzq[PPB][RB], tpn[TPA][RB], upn[FORCE ? TPA : 1][RB];
    // u starts at zero: at k = 0 its loads use the idle offset
    unsigned uoff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) uoff[r] = st.prev ? voff[r] : kIdleOffset;
    auto vload = [&](int i, int r) {
        const int zz = D::plane(i, C);
        return bload<double>(vr, vcol[r], (unsigned)(n * n) * ((zb + (unsigned)zz) % (unsigned)n) * 8u);
    };
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
        for (int a = 0; a < PPB; ++a) vzq[a][r] = a < C ? vload(a, r) : 0.0;
#pragma unroll
        for (int a = 0; a < TPA; ++a)
            tpn[a][r] = a < C ? bload<double>(slr, poff[r], (unsigned)(D::plane(a, C) * S::CC) * 8u) : 0.0;
        if constexpr (FORCE) {
#pragma unroll
            for (int a = 0; a < TPA; ++a)
                upn[a][r] = a < C ? bload<double>(ur, uoff[r], (unsigned)(D::plane(a, C) * S::CC) * 8u) : 0.0;
        }
    }
#pragma unroll
    for (int g = 0; g < C; g += PPB) {
        const int pb = PPB * ((g / PPB) & 1);
        double vz[PPB][RB], tprev[PPB][RB], uprev[PPB][RB];
#pragma unroll
        for (int h = 0; h < PPB; ++h) {
            const int i = g + h;
            if (i < C) {
                const int z = D::plane(i, C);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    vz[h][r] = vzq[i % PPB][r];
                    tprev[h][r] = tpn[i % TPA][r];
                    if (i + PPB < C) vzq[i % PPB][r] = vload(i + PPB, r);
                    if (i + TPA < C)
                        tpn[i % TPA][r] = bload<double>(slr, poff[r], (unsigned)(D::plane(i + TPA, C) * S::CC) * 8u);
                    if constexpr (FORCE) {
                        uprev[h][r] = upn[i % TPA][r];
                        if (i + TPA < C)
                            upn[i % TPA][r] =
                                bload<double>(ur, uoff[r], (unsigned)(D::plane(i + TPA, C) * S::CC) * 8u);
                    }
                    L.plane[pb + h][cl.pcw[r]] = R[r][z + D::IN];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < PPB; ++h) {
            const int i = g + h;
            if (i < C) {
                const int z = D::plane(i, C);
                const unsigned sz = (unsigned)(z * S::CC) * 8u;
                const PlaneView<C, double> pv(L.plane[0], pb + h, cl.corner);
                double yrow[2 * NO + RB];
                load_yrows_ring<C, D::IN>(pv, R, z, yrow);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const double acc = stencil_ring<C, D::IN>(pv, yrow, R[r], r, z, kw);
                    const double tz = R[r][z + D::IN];
                    const double u = acc + (vz[h][r] + st.c0) * st.invz * tz;
                    double pval[NCH];
                    double nvd = st.al * u - tprev[h][r];
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        pval[ci] = 0.0;
                        if (ci == 0 || ci < nch) {
                            pval[ci] = ch[r][ci].pv;
                            nvd += L.cs[ch[r][ci].sl()] * pval[ci];
                        }
                    }
                    if (!cl.valid(r)) nvd = 0.0;
                    R[r][z + D::OUT] = nvd;
                    bstore(tz, slr, voff[r], sz);  // t^k over t^{k-1}
                    if constexpr (FORCE) bstore(st.ua * tz + uprev[h][r] + st.uc * nvd, ur, voff[r], sz);
                    d1 += nvd * nvd;
                    d2 += nvd * tz;
                    pin(d1);
                    pin(d2);
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        if (ci == 0 || ci < nch) {
                            ch[r][ci].acc += pval[ci] * nvd;
                            pin(ch[r][ci].acc);
                        }
                    }
                    chainsd_advance<UP, C, NCH>(ch[r], snext, L.runs, pvr, z, nch);
                    if (!FORCE && z == MC && centre_r == r) {
                        mrow[st.k + 1] = nvd;
                        if (st.k == 0) L.bc[2] = nvd;
                        if (fabs(nvd) > 1.0 + A.bounds_tol) atomicOr(A.flags, kFlagBounds);
                    }
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
}

// PPB: planes per barrier of the sweeps (1 or 2).
template <int C, int NCH, int PPB>
__global__ __launch_bounds__(Shape<C>::BLOCK) void moments_ring_kernel(LaunchArgs K) {
    using S = Shape<C>;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    constexpr int NR = C + NO + 1;
    static_assert(!S::STREAM, "register ring: resident cubes only");
    __shared__ Lds<C, double, NCH> L;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    int centre_r = -1;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (cl.col[r] == MC * C + MC) centre_r = r;
    const long long slot_bytes = K.slot_elems * 8;
    const __amdgpu_buffer_rsrc_t slr =
        make_rsrc(reinterpret_cast<double *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    unsigned voff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) voff[r] = cl.valid(r) ? (unsigned)cl.col[r] * 8u : kIdleOffset;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const int npl = A.npl, half = npl / 2;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const double kin0 = -3.0 * A.w[0];

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        const double chi = uniform(A.chi[q]), zeta = uniform(A.zeta[q]);
        const double invz = uniform(1.0 / zeta);
        double kw[NO + 1];
        kw[0] = 0.0;
#pragma unroll
        for (int d = 1; d <= NO; ++d) kw[d] = uniform(-0.5 * A.w[d] * invz);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) * 8u
                                  : kIdleOffset;
        double *mrow = A.moments + q * (long long)(npl + 1);
        // t^0 = e_q in the upward sweep's input layout
        double R[RB][NR];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int z = i - (NO + 1);
                R[r][i] = (z >= 0 && centre_r == r && z == MC) ? 1.0 : 0.0;
            }
        if (tid == 0) mrow[0] = 1.0;
        int cur = 0;
        projector_dots<false>(L, pvr, cl, cur, nch, [&](int r, int z) {
            return (centre_r == r && z == MC) ? 1.0 : 0.0;
        });
        MomentsStep st;
        st.invz = invz;
        st.c0 = uniform(kin0 - chi);
        // one step; the ring layout alternates, so steps are taken in (up, down)
        // pairs and every pass of the loop starts in the upward layout
        // projector coefficients of step 0 (t^1 = Hhat t^0)
        for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK)
            L.cs[i] = i < ni ? invz * L.img_coef[i] * L.s[cur][i] : 0.0;
        __syncthreads();
        auto step = [&](int k, auto up) {
            constexpr bool UP = decltype(up)::value;
            st.al = k == 0 ? 1.0 : 2.0;
            st.k = k;
            st.prev = k > 0;
            double d[2] = {0.0, 0.0};
            moments_ring_sweep<C, NCH, UP, PPB>(A, L, cl, R, slr, vr, pvr, vcol, voff, zbase, kw, st, L.s[cur ^ 1], nch,
                                           centre_r, mrow, d[0], d[1], slr);
            // the sweep ended on a barrier: the dots of t^{k+1} are complete.
            // Coefficients of the next step, and its dot accumulator cleared;
            // the reduction's barrier publishes both.
            const double scale = uniform(2.0 * invz);
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) {
                L.cs[i] = i < ni ? scale * L.img_coef[i] * L.s[cur ^ 1][i] : 0.0;
                L.s[cur][i] = 0.0;
            }
            block_sum_once<2>(L, d, tid);
            if (k + 1 > half / 2) {
                if (tid == 0) {
                    const double r2k = 2.0 * d[0] - 1.0, r2k1 = 2.0 * d[1] - L.bc[2];
                    mrow[2 * (k + 1)] = r2k;
                    mrow[2 * (k + 1) - 1] = r2k1;
                    if (fabs(r2k) > 1.0 + A.bounds_tol || fabs(r2k1) > 1.0 + A.bounds_tol)
                        atomicOr(A.flags, kFlagBounds);
                }
            }
            cur ^= 1;
        };
        // n_pl is a multiple of 4: the number of steps, n_pl / 2, is even
        for (int k = 0; k < half; k += 2) {
            step(k, std::true_type());
            step(k + 1, std::false_type());
        }
    }
    }
}

// ---------------------------------------------------------------------------
// Nonlocal atomic forces (Sec. 3.4, nonlocal component), FP64, resident cubes:
//   f_I = -4 sum_{I' images of I} sum_q gamma h^3 p_{I'}(q) p_{I'}^T grad_{h,q} u_q,
//   u_q = sum_{j=0}^{n_pl} c_q^j t_q^j,
// for the nodes q inside some projector sphere (the other nodes add nothing).
// The recurrence runs to n_pl on the register ring with u accumulated in the
// workgroup's second buffer; then every point x of a centre image's sphere in
// the cube adds p(x) (grad_{h,q} u)(x), the gradient being the Sec. 3.1 central
// difference with legs that leave the cube dropped.
// ---------------------------------------------------------------------------
struct ForcesLds {
    double gk[kMaxForceNq];  // Fermi function at the quadrature nodes
    double cj[kMaxForceNq];  // c_q^j
    double fs[4][3];         // p^T grad u of the centre images
    double pc[4];            // p_I(q)
    int img[4];              // centre images (region slots)
    int nc;
};

// The images whose sphere contains node q (the centre column's runs that
// cover the centre plane) with p_I(q); cleared force sums.  Returns their
// number (workgroup-uniform; ends on a barrier).
template <int C, int NCH, typename AT>
__device__ int forces_centre_images(const AT &A, const Lds<C, double, NCH> &L, ForcesLds &FL, int tid) {
    constexpr int MC = (C - 1) / 2;
    if (tid == 0) {
        constexpr int cc = MC * C + MC;
        int nc = 0;
        for (int i = L.col_start[cc]; i < L.col_start[cc + 1] && i < Shape<C>::MAXRUNS; ++i) {
            const uint2 rr = L.runs[i];
            const int z0 = (int)((rr.x >> 8) & 0xFFu), z1 = (int)((rr.x >> 16) & 0xFFu);
            if (z0 <= MC && MC <= z1 && nc < 4) {
                FL.img[nc] = (int)(rr.x & 0xFFu);
                FL.pc[nc] = A.pvals[(int)rr.y + MC * A.pstride];
                ++nc;
            }
        }
        FL.nc = nc;
        for (int i = 0; i < 12; ++i) (&FL.fs[0][0])[i] = 0.0;
    }
    __syncthreads();
    return FL.nc;
}

// c_q^j, j = 0 .. n_pl, by discrete orthogonality (Sec. 3.2): the Fermi
// function at the quadrature nodes, then the coefficient table.  Ends on a
// barrier.
template <int C, typename AT>
__device__ void forces_coefficients(const AT &A, ForcesLds &FL, double chi, double zeta, int tid) {
    const int nq = A.npl + 1;
    for (int k = tid; k < nq; k += Shape<C>::BLOCK)
        FL.gk[k] = 1.0 / (1.0 + exp((zeta * A.rk[k] + chi - A.mu) / A.kT));
    __syncthreads();
    for (int j = tid; j < nq; j += Shape<C>::BLOCK) {
        double c = 0.0;
        for (int k = 0; k < nq; ++k) c += A.ctab[j * nq + k] * FL.gk[k];
        FL.cj[j] = c;
    }
    __syncthreads();
}

// p_I^T grad_{h,q} u for the centre images (one thread per run record of a
// centre image; u in cube-plane layout, complete in memory), then the forces
// -4 gamma h^3 p_I(q) (p_I^T grad u) added to the atoms.
template <int C, int NCH, typename AT>
__device__ void forces_gradient(const AT &A, const Lds<C, double, NCH> &L, ForcesLds &FL, const double *ubuf,
                                int tid) {
    using S = Shape<C>;
    const int ncent = FL.nc;
    const int nrec = L.col_start[S::CC] < S::MAXRUNS ? L.col_start[S::CC] : S::MAXRUNS;
    for (int i = tid; i < nrec; i += S::BLOCK) {
        const uint2 rr = L.runs[i];
        const int I = (int)(rr.x & 0xFFu);
        int m = -1;
        for (int mm = 0; mm < ncent; ++mm)
            if (FL.img[mm] == I) m = mm;
        if (m < 0) continue;
        int lo = 0, hi = S::CC;  // column: last c with col_start[c] <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (L.col_start[mid] <= i) lo = mid;
            else hi = mid;
        }
        const int x = lo % C, y = lo / C;
        const int z0 = (int)((rr.x >> 8) & 0xFFu), z1 = (int)((rr.x >> 16) & 0xFFu);
        double g3[3] = {0.0, 0.0, 0.0};
        for (int z = z0; z <= z1; ++z) {
            const double p = A.pvals[(int)rr.y + z * A.pstride];
            const double *uz = ubuf + (long long)z * S::CC + y * C + x;
            double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
            for (int d = 1; d <= NO; ++d) {
                const double w = A.gw[d];
                if (x + d < C) gx += w * uz[d];
                if (x - d >= 0) gx -= w * uz[-d];
                if (y + d < C) gy += w * uz[d * C];
                if (y - d >= 0) gy -= w * uz[-d * C];
                if (z + d < C) gz += w * uz[d * S::CC];
                if (z - d >= 0) gz -= w * uz[-d * S::CC];
            }
            g3[0] += p * gx;
            g3[1] += p * gy;
            g3[2] += p * gz;
        }
        atomicAdd(&FL.fs[m][0], g3[0]);
        atomicAdd(&FL.fs[m][1], g3[1]);
        atomicAdd(&FL.fs[m][2], g3[2]);
    }
    __syncthreads();
    if (tid < 3 * ncent) {
        const int m = tid / 3, ax = tid % 3, I = FL.img[m];
        atomicAdd(&A.forces[3 * L.img_atom[I] + ax], -4.0 * L.img_coef[I] * FL.pc[m] * FL.fs[m][ax]);
    }
    __syncthreads();
}


template <int C, int NCH>
__global__ __launch_bounds__(Shape<C>::BLOCK) void forces_ring_kernel(LaunchArgs K) {
    using S = Shape<C>;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    constexpr int NR = C + NO + 1;
    static_assert(!S::STREAM, "register ring: resident cubes only");
    __shared__ Lds<C, double, NCH> L;
    __shared__ ForcesLds FL;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    int centre_r = -1;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (cl.col[r] == MC * C + MC) centre_r = r;
    const long long slot_bytes = K.slot_elems * 8;
    double *ubuf = reinterpret_cast<double *>(K.wslots) + (long long)blockIdx.x * K.slot_elems;
    const __amdgpu_buffer_rsrc_t slr =
        make_rsrc(reinterpret_cast<double *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    const __amdgpu_buffer_rsrc_t ulr = make_rsrc(ubuf, slot_bytes);
    unsigned voff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) voff[r] = cl.valid(r) ? (unsigned)cl.col[r] * 8u : kIdleOffset;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const int npl = A.npl;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const double kin0 = -3.0 * A.w[0];

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        if (forces_centre_images(A, L, FL, tid) == 0) continue;
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        const double chi = uniform(A.chi[q]), zeta = uniform(A.zeta[q]);
        const double invz = uniform(1.0 / zeta);
        forces_coefficients<C>(A, FL, chi, zeta, tid);
        double kw[NO + 1];
        kw[0] = 0.0;
#pragma unroll
        for (int d = 1; d <= NO; ++d) kw[d] = uniform(-0.5 * A.w[d] * invz);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) * 8u
                                  : kIdleOffset;
        // t^0 = e_q in the upward sweep's input layout
        double R[RB][NR];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int z = i - (NO + 1);
                R[r][i] = (z >= 0 && centre_r == r && z == MC) ? 1.0 : 0.0;
            }
        int cur = 0;
        projector_dots<false>(L, pvr, cl, cur, nch, [&](int r, int z) {
            return (centre_r == r && z == MC) ? 1.0 : 0.0;
        });
        MomentsStep st;
        st.invz = invz;
        st.c0 = uniform(kin0 - chi);
        for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK)
            L.cs[i] = i < ni ? invz * L.img_coef[i] * L.s[cur][i] : 0.0;
        __syncthreads();
        auto step = [&](int k, auto up) {
            constexpr bool UP = decltype(up)::value;
            st.al = k == 0 ? 1.0 : 2.0;
            st.k = k;
            st.prev = k > 0;
            st.ua = uniform(k == 0 ? FL.cj[0] : 0.0);
            st.uc = uniform(FL.cj[k + 1]);
            double d[2] = {0.0, 0.0};
            moments_ring_sweep<C, NCH, UP, 1, true>(A, L, cl, R, slr, vr, pvr, vcol, voff, zbase, kw, st, L.s[cur ^ 1],
                                                 nch, centre_r, nullptr, d[0], d[1], ulr);
            const double scale = uniform(2.0 * invz);
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) {
                L.cs[i] = i < ni ? scale * L.img_coef[i] * L.s[cur ^ 1][i] : 0.0;
                L.s[cur][i] = 0.0;
            }
            __syncthreads();
            cur ^= 1;
        };
        // n_pl steps (t^1 .. t^{n_pl}), an even number
        for (int k = 0; k < npl; k += 2) {
            step(k, std::true_type());
            step(k + 1, std::false_type());
        }
        forces_gradient(A, L, FL, ubuf, tid);
    }
    }
}

// Nonlocal forces on the streamed cubes (wider than kResidentCube): the
// streamed recurrence of moments_kernel run to n_pl, with u accumulated in the
// third buffer.
template <int C, int NCH>
__global__ __launch_bounds__(Shape<C>::BLOCK) void forces_kernel(LaunchArgs K) {
    using S = Shape<C>;
    using T = double;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    constexpr int ZA = NO + 1;  // look-ahead of the streamed t^k
    static_assert(S::STREAM, "streamed cubes only");
    __shared__ Lds<C, T, NCH> L;
    __shared__ ForcesLds FL;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    int centre_r = -1;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (cl.col[r] == MC * C + MC) centre_r = r;
    const long long slot_bytes = K.slot_elems * 8;
    __amdgpu_buffer_rsrc_t slr =
        make_rsrc(reinterpret_cast<T *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    __amdgpu_buffer_rsrc_t sly =
        make_rsrc(reinterpret_cast<T *>(K.wslots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    double *ubuf = reinterpret_cast<double *>(K.xslots) + (long long)blockIdx.x * K.slot_elems;
    const __amdgpu_buffer_rsrc_t ulr = make_rsrc(ubuf, slot_bytes);
    unsigned voff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) voff[r] = cl.valid(r) ? (unsigned)cl.col[r] * 8u : kIdleOffset;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const int npl = A.npl;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const double kin0 = -3.0 * A.w[0];

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        if (forces_centre_images(A, L, FL, tid) == 0) continue;
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        const double chi = uniform(A.chi[q]), zeta = uniform(A.zeta[q]);
        const double invz = uniform(1.0 / zeta);
        forces_coefficients<C>(A, FL, chi, zeta, tid);
        double kw[NO + 1];
        kw[0] = 0.0;
#pragma unroll
        for (int d = 1; d <= NO; ++d) kw[d] = uniform(-0.5 * A.w[d] * invz);
        const double c0 = uniform(kin0 - chi);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) * 8u
                                  : kIdleOffset;
        T tv[RB][C];  // a window of planes of t^k
        int cur = 0;
        // t^0 goes to X here, so that every sweep reads X
        projector_dots<false>(L, pvr, cl, cur, nch, [&](int r, int z) {
            const T v = (centre_r == r && z == MC) ? 1.0 : 0.0;
            bstore(v, slr, voff[r], (unsigned)(z * S::CC) * 8u);
            return v;
        });

        for (int k = 0; k < npl; ++k) {
            const double al = k == 0 ? 1.0 : 2.0;
            const double scale = uniform(al * invz);
            const double ua = uniform(k == 0 ? FL.cj[0] : 0.0), uc = uniform(FL.cj[k + 1]);
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK)
                L.cs[i] = i < ni ? scale * L.img_coef[i] * L.s[cur][i] : 0.0;
            Chain ch[RB][NCH];
#pragma unroll
            for (int r = 0; r < RB; ++r) chains_start(L, pvr, Cols<C>::column(r), ch[r], nch);
            double *snext = L.s[cur ^ 1];
            unsigned zb = (unsigned)__builtin_amdgcn_readfirstlane((int)zbase);
            asm volatile("" : "+s"(zb));
            const bool prev = k > 0;
#pragma unroll
            for (int z = 0; z < (ZA < C ? ZA : C); ++z)
#pragma unroll
                for (int r = 0; r < RB; ++r) tv[r][z] = bload<T>(slr, voff[r], (unsigned)(z * S::CC) * 8u);
            double vzn[RB], tpn[RB], upn[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                vzn[r] = bload<T>(vr, vcol[r], (unsigned)(n * n) * (zb % (unsigned)n) * 8u);
                tpn[r] = 0.0;
                upn[r] = 0.0;
                if (prev) {
                    tpn[r] = bload<T>(sly, voff[r], 0u);
                    upn[r] = bload<T>(ulr, voff[r], 0u);
                }
            }
#pragma unroll
            for (int z = 0; z < C; ++z) {
                const unsigned sz = (unsigned)(z * S::CC) * 8u;
                double vz[RB], tprev[RB], uprev[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    vz[r] = vzn[r];
                    tprev[r] = tpn[r];
                    uprev[r] = upn[r];
                    if (z + 1 < C) {
                        const unsigned sz1 = (unsigned)((z + 1) * S::CC) * 8u;
                        const unsigned vz1 = (unsigned)(n * n) * ((zb + (unsigned)(z + 1)) % (unsigned)n) * 8u;
                        vzn[r] = bload<T>(vr, vcol[r], vz1);
                        if (prev) {
                            tpn[r] = bload<T>(sly, voff[r], sz1);
                            upn[r] = bload<T>(ulr, voff[r], sz1);
                        }
                    }
                    if (z + ZA < C) tv[r][z + ZA] = bload<T>(slr, voff[r], (unsigned)((z + ZA) * S::CC) * 8u);
                    L.plane[z & 1][cl.pcw[r]] = tv[r][z];
                }
                __syncthreads();
                const PlaneView<C, T> pv(L.plane[0], z & 1, cl.corner);
                T yrow[2 * NO + RB];
                load_yrows<C, T>(pv, tv, z, yrow);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const double acc = stencil_sum<C, T>(pv, yrow, tv[r], r, z, kw);
                    const double tz = tv[r][z];
                    const double u = acc + (vz[r] + c0) * invz * tz;
                    double pval[NCH];
                    double nvd = al * u - tprev[r];
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        pval[ci] = 0.0;
                        if (ci == 0 || ci < nch) {
                            pval[ci] = ch[r][ci].pv;
                            nvd += L.cs[ch[r][ci].sl()] * pval[ci];
                        }
                    }
                    if (!cl.valid(r)) nvd = 0.0;
                    bstore(nvd, sly, voff[r], sz);                            // t^{k+1} over t^{k-1}
                    bstore(ua * tz + uprev[r] + uc * nvd, ulr, voff[r], sz);  // u
#pragma unroll
                    for (int ci = 0; ci < NCH; ++ci) {
                        if (ci == 0 || ci < nch) {
                            ch[r][ci].acc += pval[ci] * nvd;
                            pin(ch[r][ci].acc);
                        }
                    }
                    chains_advance<C, NCH>(ch[r], snext, L.runs, pvr, z, nch);
                }
            }
            __syncthreads();
            {
                // t^k -> t^{k-1}, t^{k+1} -> t^k: X and Y swap
                const __amdgpu_buffer_rsrc_t t = slr;
                slr = sly;
                sly = t;
            }
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) L.s[cur][i] = 0.0;
            cur ^= 1;
            __syncthreads();
        }
        forces_gradient(A, L, FL, ubuf, tid);
    }
    }
}

// ---------------------------------------------------------------------------
// FP32-mixed Chebyshev moments (resident cubes).  The first kMixedFp64Steps
// steps run on the FP64 register ring (moments_ring_sweep): the early vectors
// are concentrated around q with entries of order one, and an FP32 rounding
// of them propagates into every later moment, alike for every node.  The
// remaining steps keep t^k and t^{k-1} in FP32 registers (t^{k+1} overwrites
// t^{k-1} in place; no vector moves through memory).  Every operand is
// widened before it is used and all arithmetic is FP64; the LDS plane holds
// the widened t^k, so its x and y legs need no conversion.
// ---------------------------------------------------------------------------
template <int C, int NCH, typename AT>
__device__ __forceinline__ void mixed_sweep(const AT &A, Lds<C, double, NCH> &L, const Cols<C> &cl,
                                            float (&tv)[Shape<C>::RB][C], float (&tp)[Shape<C>::RB][C],
                                            __amdgpu_buffer_rsrc_t vr, __amdgpu_buffer_rsrc_t pvr,
                                            const unsigned (&vcol)[Shape<C>::RB], unsigned zbase,
                                            const double (&kw)[NO + 1], const MomentsStep &st, double *snext,
                                            int nch, int centre_r, double *mrow, double &d1, double &d2) {
    using S = Shape<C>;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    constexpr int P = S::P;
    // The LDS plane holds the widened t^k (FP64): an FP32 plane halves the
    // LDS bytes but its x and y legs then need a conversion at every use,
    // which measured 10 % slower on the 1372-atom cell.
    using PT = double;
    double *plane = &L.plane[0][0];
    const int n = A.n;
    ChainD<true> ch[RB][NCH];
#pragma unroll
    for (int r = 0; r < RB; ++r) chainsd_start<true>(L, pvr, Cols<C>::column(r), ch[r], nch);
    unsigned zb = (unsigned)__builtin_amdgcn_readfirstlane((int)zbase);
    asm volatile("" : "+s"(zb));
    double vzn[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) vzn[r] = bload<double>(vr, vcol[r], (unsigned)(n * n) * (zb % (unsigned)n) * 8u);
#pragma unroll
    for (int z = 0; z < C; ++z) {
        double vz[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            vz[r] = vzn[r];
            if (z + 1 < C)
                vzn[r] = bload<double>(vr, vcol[r],
                                       (unsigned)(n * n) * ((zb + (unsigned)(z + 1)) % (unsigned)n) * 8u);
            plane[(z & 1) * S::PLANE + cl.pcw[r]] = (PT)tv[r][z];
        }
        __syncthreads();
        const PlaneView<C, PT> pv(plane, z & 1, cl.corner);
        PT yrow[2 * NO + RB];
#pragma unroll
        for (int j = 0; j < NO; ++j) yrow[j] = pv.ylo[j * P];
#pragma unroll
        for (int r = 0; r < RB; ++r) yrow[NO + r] = (PT)tv[r][z];
#pragma unroll
        for (int j = 0; j < NO; ++j) yrow[NO + RB + j] = pv.yhi[j * P];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            double acc[2] = {0.0, 0.0};
#pragma unroll
            for (int d = 1; d <= NO; ++d) {
                const double xs = (double)pv.xr[r * P + NO + d] + (double)pv.xr[r * P + NO - d];
                const double ys = widen_at_use(yrow[NO + r + d]) + widen_at_use(yrow[NO + r - d]);
                double zs = 0.0;
                if (z + d < C) zs = widen_at_use(tv[r][z + d]);
                if (z - d >= 0) zs = zs + widen_at_use(tv[r][z - d]);
                acc[d & 1] += kw[d] * (xs + ys + zs);
            }
            const double tz = widen_at_use(tv[r][z]);
            const double u = acc[1] + acc[0] + (vz[r] + st.c0) * st.invz * tz;
            double pval[NCH];
            double nvd = st.al * u - widen_at_use(tp[r][z]);
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci) {
                pval[ci] = 0.0;
                if (ci == 0 || ci < nch) {
                    pval[ci] = ch[r][ci].pv;
                    nvd += L.cs[ch[r][ci].sl()] * pval[ci];
                }
            }
            if (!cl.valid(r)) nvd = 0.0;
            // the moment is taken before the vector is rounded for storage
            const double moment = nvd;
            tp[r][z] = (float)nvd;  // t^{k+1} over t^{k-1}
            nvd = (double)tp[r][z];
            d1 += nvd * nvd;
            d2 += nvd * tz;
            pin(d1);
            pin(d2);
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci) {
                if (ci == 0 || ci < nch) {
                    ch[r][ci].acc += pval[ci] * nvd;
                    pin(ch[r][ci].acc);
                }
            }
            chainsd_advance<true, C, NCH>(ch[r], snext, L.runs, pvr, z, nch);
            if (z == MC && centre_r == r) {
                mrow[st.k + 1] = moment;
                if (fabs(moment) > 1.0 + A.bounds_tol) atomicOr(A.flags, kFlagBounds);
            }
        }
    }
    __syncthreads();
}

template <int C, int NCH>
__global__ __launch_bounds__(Shape<C>::BLOCK) void moments_mixed_kernel(LaunchArgs K) {
    using S = Shape<C>;
    constexpr int RB = S::RB;
    constexpr int MC = (C - 1) / 2;
    constexpr int NR = C + NO + 1;
    static_assert(!S::STREAM, "resident cubes only");
    __shared__ Lds<C, double, NCH> L;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    int centre_r = -1;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (cl.col[r] == MC * C + MC) centre_r = r;
    const long long slot_bytes = K.slot_elems * 8;
    const __amdgpu_buffer_rsrc_t slr =
        make_rsrc(reinterpret_cast<double *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    unsigned voff[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) voff[r] = cl.valid(r) ? (unsigned)cl.col[r] * 8u : kIdleOffset;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const int npl = A.npl, half = npl / 2;
    // FP64 steps: an even number (the ring sweeps come in up/down pairs)
    const int k64 = (kMixedFp64Steps < half ? kMixedFp64Steps : half) & ~1;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const double kin0 = -3.0 * A.w[0];

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        const double chi = uniform(A.chi[q]), zeta = uniform(A.zeta[q]);
        const double invz = uniform(1.0 / zeta);
        double kw[NO + 1];
        kw[0] = 0.0;
#pragma unroll
        for (int d = 1; d <= NO; ++d) kw[d] = uniform(-0.5 * A.w[d] * invz);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) * 8u
                                  : kIdleOffset;
        double *mrow = A.moments + q * (long long)(npl + 1);
        if (tid == 0) mrow[0] = 1.0;
        int cur = 0;
        projector_dots<false>(L, pvr, cl, cur, nch, [&](int r, int z) {
            return (centre_r == r && z == MC) ? 1.0 : 0.0;
        });
        MomentsStep st;
        st.invz = invz;
        st.c0 = uniform(kin0 - chi);
        // projector coefficients of step 0 (t^1 = Hhat t^0)
        for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK)
            L.cs[i] = i < ni ? invz * L.img_coef[i] * L.s[cur][i] : 0.0;
        __syncthreads();
        auto begin_step = [&](int k) {
            st.al = k == 0 ? 1.0 : 2.0;
            st.k = k;
            st.prev = k > 0;
        };
        // after a sweep (which ends on a barrier): the next step's projector
        // coefficients and cleared dot accumulator, published by the
        // reduction's barrier
        auto end_step = [&](int k, double d1, double d2) {
            const double scale = uniform(2.0 * invz);
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) {
                L.cs[i] = i < ni ? scale * L.img_coef[i] * L.s[cur ^ 1][i] : 0.0;
                L.s[cur][i] = 0.0;
            }
            double d[2] = {d1, d2};
            block_sum_once<2>(L, d, tid);
            if (k + 1 > half / 2) {
                if (tid == 0) {
                    const double r2k = 2.0 * d[0] - 1.0, r2k1 = 2.0 * d[1] - mrow[1];
                    mrow[2 * (k + 1)] = r2k;
                    mrow[2 * (k + 1) - 1] = r2k1;
                    if (fabs(r2k) > 1.0 + A.bounds_tol || fabs(r2k1) > 1.0 + A.bounds_tol)
                        atomicOr(A.flags, kFlagBounds);
                }
            }
            cur ^= 1;
        };
        // FP64 phase on the ring; t^{k-1} in the slot
        {
            double R[RB][NR];
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const int z = i - (NO + 1);
                    R[r][i] = (z >= 0 && centre_r == r && z == MC) ? 1.0 : 0.0;
                }
            for (int k = 0; k < k64; k += 2) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    begin_step(k + h);
                    double d1 = 0.0, d2 = 0.0;
                    if (h == 0)
                        moments_ring_sweep<C, NCH, true, 1>(A, L, cl, R, slr, vr, pvr, vcol, voff, zbase, kw, st,
                                                         L.s[cur ^ 1], nch, centre_r, mrow, d1, d2, slr);
                    else
                        moments_ring_sweep<C, NCH, false, 1>(A, L, cl, R, slr, vr, pvr, vcol, voff, zbase, kw, st,
                                                          L.s[cur ^ 1], nch, centre_r, mrow, d1, d2, slr);
                    end_step(k + h, d1, d2);
                }
            }
            // FP32 phase: t^k from the ring (upward input layout after an even
            // number of steps), t^{k-1} from the slot, both rounded once
            float tv[RB][C], tp[RB][C];
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int z = 0; z < C; ++z) {
                    tv[r][z] = (float)R[r][z + NO + 1];
                    tp[r][z] = k64 > 0 ? (float)bload<double>(slr, voff[r], (unsigned)(z * S::CC) * 8u) : 0.0f;
                }
            for (int k = k64; k < half; ++k) {
                begin_step(k);
                double d1 = 0.0, d2 = 0.0;
                mixed_sweep<C, NCH>(A, L, cl, tv, tp, vr, pvr, vcol, zbase, kw, st, L.s[cur ^ 1], nch, centre_r,
                                    mrow, d1, d2);
                end_step(k, d1, d2);
                // t^k -> t^{k-1}, t^{k+1} -> t^k
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int z = 0; z < C; ++z) {
                        const float t = tv[r][z];
                        tv[r][z] = tp[r][z];
                        tp[r][z] = t;
                    }
            }
        }
    }
    }
}

// ---------------------------------------------------------------------------
// Lanczos bounds on the register ring, one pass per step (Sec. 3.2; Paige's
// ordering up to rounding).  x_j denotes w_{j-1} = beta_{j-1} v_j, kept
// unnormalised (x_0 = v_0, the start vector); sigma_j = 1 / beta_{j-1}.
// Sweep j:
//   * forms x_j plane by plane NO planes ahead of the stencil, in the ring:
//       x_j = sigma_{j-1} (U_{j-1} + sum_I c_I s_I(x_{j-1}) p_I)
//             - beta_{j-2} sigma_{j-2} x_{j-2} - alpha_{j-1} sigma_{j-1} x_{j-1}
//     with U_{j-1} = L x_{j-1} the local (stencil + potential) part from the
//     previous sweep, x_{j-1} and x_{j-2} read from the two workgroup slots;
//     x_j is written over x_{j-2}; the same walk over the projector runs adds
//     the projector term and accumulates s_I(x_j) = p_I . x_j;
//   * applies the local part: U_j = L x_j into the ring's output layout.
// After the sweep: beta_{j-1} = |x_j|,
//   alpha_j = sigma_j^2 (x_j . U_j + sum_I c_I s_I(x_j)^2) - sigma_{j-1} x_{j-1} . x_j,
// which is u_j . v_j with u_j = H v_j - beta_{j-1} v_{j-1}.
// Three vector transfers per step (read x_{j-1}, x_{j-2}; write x_j).
// ---------------------------------------------------------------------------
struct LanczosStep {
    int j;
    double fu, fa, fb;  // formation coefficients of U_{j-1} (+ projector part), x_{j-1}, x_{j-2}
    bool ra, rb;        // x_{j-1} / x_{j-2} are read
};

template <int C, int NCH, bool UP, int PPB, typename AT>
__device__ __forceinline__ void lanczos_ring_sweep(const AT &A, Lds<C, double, NCH> &L, const Cols<C> &cl,
                                                   double (&R)[Shape<C>::RB][C + NO + 1],
                                                   __amdgpu_buffer_rsrc_t rda, __amdgpu_buffer_rsrc_t rdb,
                                                   __amdgpu_buffer_rsrc_t vr, __amdgpu_buffer_rsrc_t pvr,
                                                   const unsigned (&vcol)[Shape<C>::RB],
                                                   unsigned tslot, unsigned zbase,
                                                   const double (&kw)[NO + 1], double kin0, const LanczosStep &st,
                                                   double *snext, int nch, double (&dots)[4]) {
    using S = Shape<C>;
    using D = RingDir<UP>;
    constexpr int RB = S::RB;
    constexpr int FA = kLanczosAhead;  // slot reads run FA planes ahead of the formation
    const int n = A.n;
    ChainD<UP> ch[RB][NCH];
#pragma unroll
    for (int r = 0; r < RB; ++r) chainsd_start<UP>(L, pvr, Cols<C>::column(r), ch[r], nch);
    unsigned zb = (unsigned)__builtin_amdgcn_readfirstlane((int)zbase);
    asm volatile("" : "+s"(zb));
    // slots not yet written in this node are not read (their loads return 0)
    const unsigned aoff = st.ra ? tslot : kIdleOffset;
    const unsigned boff = st.rb ? tslot : kIdleOffset;
    double an[FA][RB], bn[FA][RB];
#pragma unroll
    for (int f = 0; f < FA; ++f) {
        if (f < C) {
            const unsigned so = (unsigned)(D::plane(f, C) * S::SP) * 8u;
            slot_load<RB>(an[f], rda, aoff, so);
            slot_load<RB>(bn[f], rdb, boff, so);
        }
    }
    double da = 0.0, db = 0.0, de = 0.0;
    // formation of plane D::plane(f): x into the ring's input layout and the slot
    auto form = [&](int f) {
        const int z = D::plane(f, C);
        const unsigned sz = (unsigned)(z * S::SP) * 8u;
        double av[RB], bv[RB], xs[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            av[r] = an[f % FA][r];
            bv[r] = bn[f % FA][r];
        }
        if (f + FA < C) {
            const unsigned so = (unsigned)(D::plane(f + FA, C) * S::SP) * 8u;
            slot_load<RB>(an[f % FA], rda, aoff, so);
            slot_load<RB>(bn[f % FA], rdb, boff, so);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const double a = av[r], b = bv[r];
            // step 0: fu = 1, fa = fb = 0 and no projector coefficients, so x_0
            // passes through unchanged
            double pu = R[r][z + D::IN];
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci)
                if (ci == 0 || ci < nch) pu += L.cs[ch[r][ci].sl()] * ch[r][ci].pv;
            double x = st.fu * pu - st.fb * b - st.fa * a;
            if (!cl.valid(r)) x = 0.0;
            R[r][z + D::IN] = x;
            xs[r] = x;
            db += x * x;
            de += x * a;
            pin(db);
            pin(de);
#pragma unroll
            for (int ci = 0; ci < NCH; ++ci) {
                if (ci == 0 || ci < nch) {
                    ch[r][ci].acc += ch[r][ci].pv * x;
                    pin(ch[r][ci].acc);
                }
            }
            chainsd_advance<UP, C, NCH>(ch[r], snext, L.runs, pvr, z, nch);
        }
        slot_store<RB>(xs, rdb, tslot, sz);  // x_j over x_{j-2}
    };
#pragma unroll
    for (int f = 0; f < NO && f < C; ++f) form(f);
    // PPB planes share one barrier; V_eff runs PPB planes ahead
    static_assert(PPB == 1 || PPB == 2, "one or two planes per barrier");
    double vzq[PPB][RB];
    auto vload = [&](int i, int r) {
        const int zz = D::plane(i, C);
        return bload<double>(vr, vcol[r], (unsigned)(n * n) * ((zb + (unsigned)zz) % (unsigned)n) * 8u);
    };
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int a = 0; a < PPB; ++a) vzq[a][r] = a < C ? vload(a, r) : 0.0;
#pragma unroll
    for (int g = 0; g < C; g += PPB) {
        const int pb = PPB * ((g / PPB) & 1);
        double vz[PPB][RB];
#pragma unroll
        for (int h = 0; h < PPB; ++h) {
            const int i = g + h;
            if (i < C) {
                const int z = D::plane(i, C);
                if (i + NO < C) form(i + NO);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    vz[h][r] = vzq[i % PPB][r];
                    if (i + PPB < C) vzq[i % PPB][r] = vload(i + PPB, r);
                    L.plane[pb + h][cl.pcw[r]] = R[r][z + D::IN];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < PPB; ++h) {
            const int i = g + h;
            if (i < C) {
                const int z = D::plane(i, C);
                const PlaneView<C, double> pv(L.plane[0], pb + h, cl.corner);
                double yrow[2 * NO + RB];
                load_yrows_ring<C, D::IN>(pv, R, z, yrow);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const double xz = R[r][z + D::IN];
                    double u = stencil_ring<C, D::IN>(pv, yrow, R[r], r, z, kw) + (vz[h][r] + kin0) * xz;
                    if (!cl.valid(r)) u = 0.0;
                    R[r][z + D::OUT] = u;
                    da += u * xz;
                    pin(da);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    dots[0] = da;
    dots[1] = db;
    dots[2] = de;
}

// PPB: planes per barrier of the sweeps (1 or 2).
template <int C, int NCH, int PPB>
__global__ __launch_bounds__(Shape<C>::BLOCK) void lanczos_ring_kernel(LaunchArgs K) {
    using S = Shape<C>;
    constexpr int RB = S::RB;
    constexpr int NR = C + NO + 1;
    static_assert(!S::STREAM, "register ring: resident cubes only");
    __shared__ Lds<C, double, NCH> L;
    __shared__ LanczosLds LL;
    const int tid = threadIdx.x;
    Cols<C> cl;
    cl.init(tid);
    const long long slot_bytes = K.slot_elems * 8;
    // x_j goes to slot j % 2
    const __amdgpu_buffer_rsrc_t s0 =
        make_rsrc(reinterpret_cast<double *>(K.slots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    const __amdgpu_buffer_rsrc_t s1 =
        make_rsrc(reinterpret_cast<double *>(K.wslots) + (long long)blockIdx.x * K.slot_elems, slot_bytes);
    const long long ns = (long long)C * C * C;

    WorkSource work;
    SnapPtr Ap;
    long long qfirst, qend, qstep;
    while (work.next(K, L, tid, Ap, qfirst, qend, qstep)) {
    const auto &A = *Ap;
    const int n = A.n;
    const __amdgpu_buffer_rsrc_t vr = make_rsrc(A.veff, A.nd * 8);
    const __amdgpu_buffer_rsrc_t pvr = make_rsrc(A.pvals, A.pvals_bytes);
    const int kmax = (long long)A.n_lanczos < ns ? A.n_lanczos : (int)ns;
    const double rnorm = 1.0 / A.start_norm;

    for (long long q = qfirst; q < qend; q += qstep) {
        int qi, qj, qk;
        node_coords(q, n, qi, qj, qk);
        setup_region(A, L, qi, qj, qk, tid);
        const int ni = L.ni < kMaxImages ? L.ni : kMaxImages;
        const int nch = L.nch;
        const unsigned zbase = (unsigned)pmod(qk - A.m, n);
        double kw[NO + 1];
        kw[0] = 0.0;
#pragma unroll
        for (int d = 1; d <= NO; ++d) kw[d] = uniform(-0.5 * A.w[d]);
        const double kin0 = uniform(-3.0 * A.w[0]);
        unsigned vcol[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            vcol[r] = cl.valid(r) ? (unsigned)(pmod(qi - A.m + cl.x, n) + n * pmod(qj - A.m + cl.y0 + r, n)) * 8u
                                  : kIdleOffset;
        // x_0 = v_0[a] = (u(a) - 1/2) / |u - 1/2|, a = local cube index, in the
        // upward sweep's input layout
        double R[RB][NR];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int z = i - (NO + 1);
                R[r][i] = (z >= 0 && cl.valid(r))
                              ? (unit_from_seed((unsigned long long)(cl.col[r] + C * C * z)) - 0.5) * rnorm
                              : 0.0;
            }
        for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) L.cs[i] = 0.0;
        int cur = 0;  // L.s[cur]: dots of x_{j-1}; L.s[cur ^ 1] receives those of x_j
        double sig_m1 = 1.0, sig_m2 = 0.0;  // sigma_{j-1}, sigma_{j-2}
        double al_m1 = 0.0, be_m2 = 0.0;    // alpha_{j-1}, beta_{j-2}
        double gersh = 0.0;
        int ksteps = kmax;
        __syncthreads();
        // one step; returns false when the recurrence ends.  The ring layout
        // alternates, so steps are taken in (up, down) pairs and every pass of
        // the loop starts in the upward layout.
        auto step = [&](int j, auto up) -> bool {
            constexpr bool UP = decltype(up)::value;
            LanczosStep st;
            st.j = j;
            st.fu = uniform(sig_m1);
            st.fa = uniform(al_m1 * sig_m1);
            st.fb = uniform(be_m2 * sig_m2);
            st.ra = j >= 1;
            st.rb = j >= 2;
            const __amdgpu_buffer_rsrc_t rda = (j & 1) ? s0 : s1;  // x_{j-1}
            const __amdgpu_buffer_rsrc_t rdb = (j & 1) ? s1 : s0;  // x_{j-2}, then x_j
            double dots[4];
            lanczos_ring_sweep<C, NCH, UP, PPB>(A, L, cl, R, rda, rdb, vr, pvr, vcol, cl.slot, zbase, kw, kin0, st,
                                           L.s[cur ^ 1], nch, dots);
            // the sweep ended on a barrier: every run is closed.  sum_I c_I
            // s_I(x_j)^2, the next formation's coefficients c_I s_I(x_j) and a
            // cleared accumulator for its dots (published by the reduction's
            // barrier)
            double dimg = 0.0;
            for (int i = fresh_tid(); i < kMaxImages; i += S::BLOCK) {
                const double sj = L.s[cur ^ 1][i];
                if (i < ni) dimg += L.img_coef[i] * sj * sj;
                L.cs[i] = i < ni ? L.img_coef[i] * sj : 0.0;
                L.s[cur][i] = 0.0;
            }
            dots[3] = dimg;
            block_sum_once<4>(L, dots, tid);
            double sig = 1.0;
            if (j >= 1) {
                const double be = uniform(sqrt(dots[1]));  // beta_{j-1}
                gersh = fmax(gersh, fabs(al_m1) + be + be_m2);
                if (tid == 0) {
                    LL.be[j - 1] = be;
                    if (!isfinite(be)) atomicOr(A.flags, kFlagLanczos);
                }
                if (be <= 1e-13 * gersh) {
                    ksteps = j;
                    return false;
                }
                sig = uniform(1.0 / be);
                be_m2 = be;
            }
            const double al = j >= 1 ? uniform(sig * sig * (dots[0] + dots[3]) - sig_m1 * dots[2])
                                     : uniform(dots[0] + dots[3]);
            if (tid == 0) {
                LL.al[j] = al;
                if (!isfinite(al)) atomicOr(A.flags, kFlagLanczos);
            }
            if (j == kmax - 1) return false;
            cur ^= 1;
            sig_m2 = sig_m1;
            sig_m1 = sig;
            al_m1 = al;
            return true;
        };
        for (int j = 0; j < kmax; j += 2) {
            if (!step(j, std::true_type())) break;
            if (!step(j + 1, std::false_type())) break;
        }
        __syncthreads();
        if (tid < 64) sturm_extremes(ksteps, LL.al, LL.be, L.bc, tid);
        __syncthreads();
        if (tid == 0) {
            const double lmn = L.bc[0], lmx = L.bc[1];
            if (A.lmin) A.lmin[q] = lmn;
            if (A.lmax) A.lmax[q] = lmx;
            A.chi[q] = 0.5 * (lmx + lmn);
            A.zeta[q] = (1.0 + A.margin) * 0.5 * (lmx - lmn);
        }
        __syncthreads();
    }
    }
}

#if defined(SQ_COMMON_ONLY) || !defined(SQ_CUBES)
// ---------------------------------------------------------------------------
// Fermi level, density and energies (Sec. 3.2-3.3).  The Chebyshev sums are
// regrouped through per-node quadrature weights
//   W_qk = sum_j c-table[j][k] rho_q^j,  c-table[j][k] = (2 - delta_j0)/N_q cos(j theta_k),
// so that sum_j c_q^j rho_q^j = sum_k g(lambda_qk) W_qk with
// lambda_qk = zeta_q r_k + chi_q (same quadrature, regrouped).
// ---------------------------------------------------------------------------
__global__ void set_bounds_kernel(const double *lmin, const double *lmax, double *chi, double *zeta,
                                  long long nd, double margin) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nd;
         q += (long long)gridDim.x * blockDim.x) {
        chi[q] = 0.5 * (lmax[q] + lmin[q]);
        zeta[q] = (1.0 + margin) * 0.5 * (lmax[q] - lmin[q]);
    }
}

// Fill of int counters (a kernel, not a memset, so that it can sit in a
// captured graph).
__global__ void zero_ints_kernel(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void zero_doubles_kernel(double *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

__global__ void weights_kernel(const double *mom, const double *ctab, double *W, long long nd, int npl) {
    const int nq = npl + 1;
    const long long total = nd * nq;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long q = i / nq;
        const int k = (int)(i - q * nq);
        const double *r = mom + q * nq;
        double s = 0.0;
        for (int j = 0; j < nq; ++j) s += ctab[j * nq + k] * r[j];
        W[i] = s;
    }
}

__device__ __forceinline__ double fermi_fn(double x) { return 1.0 / (1.0 + exp(x)); }

__device__ __forceinline__ double entropy_fn(double x) {
    const double ax = fabs(x), e = exp(-ax);
    return -(log1p(e) + ax * e / (1.0 + e));
}

constexpr int kRedBlock = 256;

__device__ __forceinline__ double block_reduce(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kRedBlock / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kRedBlock) void extent_kernel(const double *chi, const double *zeta,
                                                           long long nd, double *partials) {
    __shared__ double sh[kRedBlock / 64];
    double lo = INFINITY, hi = -INFINITY;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nd;
         q += (long long)gridDim.x * blockDim.x) {
        lo = fmin(lo, chi[q] - zeta[q]);
        hi = fmax(hi, chi[q] + zeta[q]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    __shared__ double sh2[kRedBlock / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = lo;
        sh2[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < kRedBlock / 64; ++i) {
            lo = fmin(lo, sh[i]);
            hi = fmax(hi, sh2[i]);
        }
        partials[2 * blockIdx.x] = lo;
        partials[2 * blockIdx.x + 1] = hi;
    }
}

// min and max of a - b (b may be null: of a) per block, for extent_final.
__global__ __launch_bounds__(kRedBlock) void diff_extent_kernel(const double *a, const double *b, long long n,
                                                                double *partials) {
    __shared__ double sh[kRedBlock / 64], sh2[kRedBlock / 64];
    double lo = INFINITY, hi = -INFINITY;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double d = b ? a[i] - b[i] : a[i];
        lo = fmin(lo, d);
        hi = fmax(hi, d);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = lo;
        sh2[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < kRedBlock / 64; ++i) {
            lo = fmin(lo, sh[i]);
            hi = fmax(hi, sh2[i]);
        }
        partials[2 * blockIdx.x] = lo;
        partials[2 * blockIdx.x + 1] = hi;
    }
}

__global__ void extent_final(const double *partials, int nblk, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double lo = INFINITY, hi = -INFINITY;
        for (int i = 0; i < nblk; ++i) {
            lo = fmin(lo, partials[2 * i]);
            hi = fmax(hi, partials[2 * i + 1]);
        }
        out[0] = lo;
        out[1] = hi;
    }
}

__global__ __launch_bounds__(kRedBlock) void count_kernel(const double *W, const double *chi,
                                                          const double *zeta, const double *rk,
                                                          long long nd, int nq, double mu, double kT,
                                                          double *partials) {
    __shared__ double sh[kRedBlock / 64];
    const long long total = nd * nq;
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long q = i / nq;
        const int k = (int)(i - q * nq);
        const double lam = zeta[q] * rk[k] + chi[q];
        acc += fermi_fn((lam - mu) / kT) * W[i];
    }
    const double s = block_reduce(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// N(mu_eval) of every snapshot whose Brent search is pending (blockIdx.y =
// snapshot); per snapshot the same partial sums as count_kernel.
__global__ __launch_bounds__(kRedBlock) void count_batch_kernel(const FermiSnap *fs, const BrentState *st,
                                                                double *partials) {
    __shared__ double sh[kRedBlock / 64];
    const int si = blockIdx.y;
    const int ph = st[si].phase;
    if (ph < kBrentLow || ph > kBrentIterate) return;
    const FermiSnap f = fs[si];
    const double mu = st[si].mu_eval;
    const long long total = f.nd * f.nq;
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long q = i / f.nq;
        const int k = (int)(i - q * f.nq);
        const double lam = f.zeta[q] * f.rk[k] + f.chi[q];
        acc += fermi_fn((lam - mu) / f.kT) * f.W[i];
    }
    const double s = block_reduce(acc, sh);
    if (threadIdx.x == 0) partials[(long long)si * gridDim.x + blockIdx.x] = s;
}

__global__ void brent_begin_kernel(BrentState *st, const BrentParams *prm, const double *ext, int nsnap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsnap) return;
    const BrentParams p = prm[i];
    BrentState b;
    brent_begin(b, ext[2 * i], ext[2 * i + 1], p.kT, p.n_e, p.xtol, p.ftol, p.max_it);
    st[i] = b;
}

// One Brent step per snapshot from the fixed-order sum of its partials
// (N = 2 sum_q sum_k g(lambda_qk) W_qk).
__global__ void brent_feed_kernel(BrentState *st, const double *partials, int nblk, int nsnap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsnap) return;
    BrentState b = st[i];
    if (b.phase < kBrentLow || b.phase > kBrentIterate) return;
    double sum = 0.0;
    for (int j = 0; j < nblk; ++j) sum += partials[(long long)i * nblk + j];
    brent_feed(b, 2.0 * sum);  // two electrons per state
    st[i] = b;
}

__global__ __launch_bounds__(kRedBlock) void density_kernel(const double *W, const double *chi,
                                                            const double *zeta, const double *rk,
                                                            long long nd, int nq, double mu_arg,
                                                            const double *mu_dev, double kT, double h3,
                                                            double *rho, double *partials) {
    __shared__ double sh[kRedBlock / 64];
    const double mu = mu_dev ? *mu_dev : mu_arg;
    double eb = 0.0, en = 0.0, er = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nd;
         q += (long long)gridDim.x * blockDim.x) {
        const double c = chi[q], z = zeta[q];
        const double *w = W + q * nq;
        double sg = 0.0, sb = 0.0, se = 0.0;
        for (int k = 0; k < nq; ++k) {
            const double lam = z * rk[k] + c;
            const double x = (lam - mu) / kT;
            const double g = fermi_fn(x);
            sg += g * w[k];
            sb += lam * g * w[k];
            se += entropy_fn(x) * w[k];
        }
        const double r = 2.0 / h3 * sg;
        rho[q] = r;
        eb += 2.0 * sb;
        en += 2.0 * kT * se;
        er += r;
    }
    const double a = block_reduce(eb, sh);
    const double b = block_reduce(en, sh);
    const double c = block_reduce(er, sh);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = a;
        partials[3 * blockIdx.x + 1] = b;
        partials[3 * blockIdx.x + 2] = c;
    }
}

// Fixed-order sum of `width` interleaved partial arrays (deterministic).
__global__ void sum_partials(const double *partials, int nblk, int width, double *out) {
    const int j = threadIdx.x;
    if (blockIdx.x == 0 && j < width) {
        double s = 0.0;
        for (int i = 0; i < nblk; ++i) s += partials[width * i + j];
        out[j] = s;
    }
}

// Density and energies straight from the moments, for the allocation-free
// entry point: the quadrature weights W_qk = sum_j c-table[j][k] rho_q^j of a
// node are formed in registers (same sums, same order as weights_kernel), so
// no N_d x N_q buffer is needed.  Per-block partials go to `partials`.
__global__ __launch_bounds__(kRedBlock) void density_direct_kernel(const double *mom, const double *ctab,
                                                                   const double *chi, const double *zeta,
                                                                   const double *rk, long long nd, int nq,
                                                                   double mu, double kT, double h3, double *rho,
                                                                   double *partials) {
    __shared__ double sh[kRedBlock / 64];
    double eb = 0.0, en = 0.0, er = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nd;
         q += (long long)gridDim.x * blockDim.x) {
        const double c = chi[q], z = zeta[q];
        const double *r = mom + q * nq;
        double sg = 0.0, sb = 0.0, se = 0.0;
        for (int k = 0; k < nq; ++k) {
            double w = 0.0;
            for (int j = 0; j < nq; ++j) w += ctab[j * nq + k] * r[j];
            const double lam = z * rk[k] + c;
            const double x = (lam - mu) / kT;
            const double g = fermi_fn(x);
            sg += g * w;
            sb += lam * g * w;
            se += entropy_fn(x) * w;
        }
        const double rq = 2.0 / h3 * sg;
        rho[q] = rq;
        eb += 2.0 * sb;
        en += 2.0 * kT * se;
        er += rq;
    }
    const double a = block_reduce(eb, sh);
    const double b = block_reduce(en, sh);
    const double c = block_reduce(er, sh);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = a;
        partials[3 * blockIdx.x + 1] = b;
        partials[3 * blockIdx.x + 2] = c;
    }
}

// Device scratch of the allocation-free density entry point: the per-block
// partials of the reduction followed by the three reduced sums.  Its size does
// not depend on the cell (the reduction uses at most kStaticBlocks blocks).
// One copy per GPU, alive until the process ends.
constexpr int kStaticBlocks = 1024;
constexpr int kStaticScratchDoubles = 3 * kStaticBlocks + 4;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

#endif  // common part

}  // namespace

#define SQ_ALL_CUBES X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29) X(31) X(33) X(35) X(37)

#ifndef SQ_COMMON_ONLY
// Launchers.  Resident cubes (up to kResidentCube) run the register-ring
// kernels in FP64 and moments_mixed_kernel in FP32-mixed mode, built for
// 1, 2 or 4 projector chains.  Streamed cubes are built with two chains only
// (the host rejects deeper sphere overlaps there) and run the FP64 streamed
// kernels in both precisions: with the current vector streamed through
// memory, FP32 storage saves no registers, and its operand widening made the
// mixed kernel slower than the FP64 one there.
template <int c, typename F>
hipError_t with_chains(int nch, F &&f) {
    if constexpr (!Shape<c>::STREAM) {
        if (nch <= 1) return f(std::integral_constant<int, 1>());
        if (nch <= 2) return f(std::integral_constant<int, 2>());
        if (nch <= 4) return f(std::integral_constant<int, 4>());
        return hipErrorInvalidValue;
    } else {
        if (nch <= 2) return f(std::integral_constant<int, 2>());
        return hipErrorInvalidValue;
    }
}
// Planes per barrier of the ring kernels for shape bits `shape`.
template <int c, typename F>
hipError_t with_planes(int shape, F &&f) {
    if constexpr (has_two_plane_shape(c))
        if (shape & kShapeTwoPlanes) return f(std::integral_constant<int, 2>());
    return f(std::integral_constant<int, 1>());
}
template <int c>
hipError_t launch_lanczos_t(const LaunchArgs &a, int nch, int nwg, hipStream_t s, int shape) {
    return with_chains<c>(nch, [&](auto ncht) {
        constexpr int NCH = decltype(ncht)::value;
        if constexpr (!Shape<c>::STREAM) {
            return with_planes<c>(shape, [&](auto ppbt) {
                constexpr int PPB = decltype(ppbt)::value;
                hipLaunchKernelGGL((lanczos_ring_kernel<c, NCH, PPB>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
                return hipGetLastError();
            });
        } else {
            hipLaunchKernelGGL((lanczos_kernel<c, NCH>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
            return hipGetLastError();
        }
    });
}
// The FP32-mixed moments kernel has one plane per barrier (the two-plane bit
// selects the FP64 moments sweep's variant only).
template <int c>
hipError_t launch_moments_t(const LaunchArgs &a, int nch, bool mixed, int nwg, hipStream_t s, int shape) {
    return with_chains<c>(nch, [&](auto ncht) {
        constexpr int NCH = decltype(ncht)::value;
        if constexpr (!Shape<c>::STREAM) {
            if (mixed) {
                hipLaunchKernelGGL((moments_mixed_kernel<c, NCH>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
                return hipGetLastError();
            }
            return with_planes<c>(shape, [&](auto ppbt) {
                constexpr int PPB = decltype(ppbt)::value;
                hipLaunchKernelGGL((moments_ring_kernel<c, NCH, PPB>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
                return hipGetLastError();
            });
        } else {
            hipLaunchKernelGGL((moments_kernel<c, NCH>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
            return hipGetLastError();
        }
    });
}
#if !SQ_TWO_ROWS
template <int c>
hipError_t launch_forces_t(const LaunchArgs &a, int nch, int nwg, hipStream_t s) {
    if constexpr (!Shape<c>::STREAM) {
        return with_chains<c>(nch, [&](auto ncht) {
            constexpr int NCH = decltype(ncht)::value;
            hipLaunchKernelGGL((forces_ring_kernel<c, NCH>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
            return hipGetLastError();
        });
    } else {
        return with_chains<c>(nch, [&](auto ncht) {
            constexpr int NCH = decltype(ncht)::value;
            hipLaunchKernelGGL((forces_kernel<c, NCH>), dim3(nwg), dim3(Shape<c>::BLOCK), 0, s, a);
            return hipGetLastError();
        });
    }
}
#endif
template <int c>
hipError_t occupancy_t(bool lanczos, bool mixed, int nch, int *nb, int shape) {
    const int B = Shape<c>::BLOCK;
    return with_chains<c>(nch, [&](auto ncht) {
        constexpr int NCH = decltype(ncht)::value;
        if constexpr (!Shape<c>::STREAM) {
            if (!lanczos && mixed) return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, moments_mixed_kernel<c, NCH>, B, 0);
            return with_planes<c>(shape, [&](auto ppbt) {
                constexpr int PPB = decltype(ppbt)::value;
                if (lanczos)
                    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, lanczos_ring_kernel<c, NCH, PPB>, B, 0);
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, moments_ring_kernel<c, NCH, PPB>, B, 0);
            });
        } else {
            if (lanczos) return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, lanczos_kernel<c, NCH>, B, 0);
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, moments_kernel<c, NCH>, B, 0);
        }
    });
}

// Per-cube entry points of this translation unit (SQ_CUBES lists its cubes;
// the two-row build has no force kernels).
#define X_RECURRENCE(c)                                                                                     \
    hipError_t lanczos_c##c(const LaunchArgs &a, int nch, int nwg, hipStream_t s, int shape) {              \
        return launch_lanczos_t<c>(a, nch, nwg, s, shape);                                                  \
    }                                                                                                       \
    hipError_t moments_c##c(const LaunchArgs &a, int nch, bool mixed, int nwg, hipStream_t s, int shape) { \
        return launch_moments_t<c>(a, nch, mixed, nwg, s, shape);                                           \
    }                                                                                                       \
    hipError_t occupancy_c##c(bool lanczos, bool mixed, int nch, int *nb, int shape) {                      \
        return occupancy_t<c>(lanczos, mixed, nch, nb, shape);                                              \
    }                                                                                                       \
    int block_c##c() { return Shape<c>::BLOCK; }
#if SQ_TWO_ROWS
#define X(c) X_RECURRENCE(c)
#else
#define X(c)                                                                       \
    X_RECURRENCE(c)                                                                \
    hipError_t forces_c##c(const LaunchArgs &a, int nch, int nwg, hipStream_t s) { \
        return launch_forces_t<c>(a, nch, nwg, s);                                 \
    }
#endif
#ifdef SQ_CUBES
SQ_CUBES
#else
SQ_ALL_CUBES
#endif
#undef X
#undef X_RECURRENCE
#endif  // !SQ_COMMON_ONLY

#if SQ_TWO_ROWS
}  // namespace two_rows
#endif

#if defined(SQ_COMMON_ONLY) || !defined(SQ_CUBES)
#define X_RECURRENCE_DECL(c)                                                                               \
    hipError_t lanczos_c##c(const LaunchArgs &a, int nch, int nwg, hipStream_t s, int shape);              \
    hipError_t moments_c##c(const LaunchArgs &a, int nch, bool mixed, int nwg, hipStream_t s, int shape); \
    hipError_t occupancy_c##c(bool lanczos, bool mixed, int nch, int *nb, int shape);                      \
    int block_c##c();
#define X(c)          \
    X_RECURRENCE_DECL(c) \
    hipError_t forces_c##c(const LaunchArgs &a, int nch, int nwg, hipStream_t s);
SQ_ALL_CUBES
#undef X
// cubes with a two-row build (has_two_row_shape)
#define SQ_TWO_ROW_CUBES X(21) X(23) X(25) X(27)
namespace two_rows {
#define X(c) X_RECURRENCE_DECL(c)
SQ_TWO_ROW_CUBES
#undef X
}  // namespace two_rows
#undef X_RECURRENCE_DECL

int recurrence_block(int C, int shape) {
    if (shape & ~shape_variants(C)) return 0;
    if (shape & kShapeTwoRows) {
        switch (C) {
#define X(c) case c: return two_rows::block_c##c();
            SQ_TWO_ROW_CUBES
#undef X
            default: return 0;
        }
    }
    switch (C) {
#define X(c) case c: return block_c##c();
        SQ_ALL_CUBES
#undef X
        default: return 0;
    }
}

hipError_t recurrence_occupancy(int C, bool lanczos, bool mixed, int nch, int *blocks_per_cu, int shape) {
    if (shape & ~shape_variants(C)) return hipErrorInvalidValue;
    if (shape & kShapeTwoRows) {
        switch (C) {
#define X(c) case c: return two_rows::occupancy_c##c(lanczos, mixed, nch, blocks_per_cu, shape);
            SQ_TWO_ROW_CUBES
#undef X
            default: return hipErrorInvalidValue;
        }
    }
    switch (C) {
#define X(c) case c: return occupancy_c##c(lanczos, mixed, nch, blocks_per_cu, shape);
        SQ_ALL_CUBES
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lanczos(const LaunchArgs &a, int C, int nch, int nwg, hipStream_t s, int shape) {
    if (shape & ~shape_variants(C)) return hipErrorInvalidValue;
    if (shape & kShapeTwoRows) {
        switch (C) {
#define X(c) case c: return two_rows::lanczos_c##c(a, nch, nwg, s, shape);
            SQ_TWO_ROW_CUBES
#undef X
            default: return hipErrorInvalidValue;
        }
    }
    switch (C) {
#define X(c) case c: return lanczos_c##c(a, nch, nwg, s, shape);
        SQ_ALL_CUBES
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_moments(const LaunchArgs &a, int C, int nch, bool mixed, int nwg, hipStream_t s, int shape) {
    if (shape & ~shape_variants(C)) return hipErrorInvalidValue;
    if (shape & kShapeTwoRows) {
        switch (C) {
#define X(c) case c: return two_rows::moments_c##c(a, nch, mixed, nwg, s, shape);
            SQ_TWO_ROW_CUBES
#undef X
            default: return hipErrorInvalidValue;
        }
    }
    switch (C) {
#define X(c) case c: return moments_c##c(a, nch, mixed, nwg, s, shape);
        SQ_ALL_CUBES
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forces(const LaunchArgs &a, int C, int nch, int nwg, hipStream_t s) {
    switch (C) {
#define X(c) case c: return forces_c##c(a, nch, nwg, s);
        SQ_ALL_CUBES
#undef X
        default: return hipErrorInvalidValue;
    }
}

namespace {
static int grid_for(long long work, int block) {
    long long g = (work + block - 1) / block;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_set_bounds(const double *lmin, const double *lmax, double *chi, double *zeta,
                             long long nd, double margin, hipStream_t s) {
    hipLaunchKernelGGL(set_bounds_kernel, dim3(grid_for(nd, 256)), dim3(256), 0, s, lmin, lmax, chi, zeta,
                       nd, margin);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_doubles(double *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_doubles_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_quadrature_weights(const double *mom, const double *ctab, double *W, long long nd,
                                     int npl, hipStream_t s) {
    hipLaunchKernelGGL(weights_kernel, dim3(grid_for(nd * (npl + 1), 256)), dim3(256), 0, s, mom, ctab, W,
                       nd, npl);
    return hipGetLastError();
}

hipError_t launch_diff_extent(const double *a, const double *b, long long n, double *partials, int nblk,
                              double *out, hipStream_t s) {
    hipLaunchKernelGGL(diff_extent_kernel, dim3(nblk), dim3(kRedBlock), 0, s, a, b, n, partials);
    hipLaunchKernelGGL(extent_final, dim3(1), dim3(64), 0, s, partials, nblk, out);
    return hipGetLastError();
}

hipError_t launch_extent(const double *chi, const double *zeta, long long nd, double *partials, int nblk,
                         double *out, hipStream_t s) {
    hipLaunchKernelGGL(extent_kernel, dim3(nblk), dim3(kRedBlock), 0, s, chi, zeta, nd, partials);
    hipLaunchKernelGGL(extent_final, dim3(1), dim3(64), 0, s, partials, nblk, out);
    return hipGetLastError();
}

hipError_t launch_count(const double *W, const double *chi, const double *zeta, const double *rk,
                        long long nd, int nq, double mu, double kT, double *partials, int nblk, double *out,
                        hipStream_t s) {
    hipLaunchKernelGGL(count_kernel, dim3(nblk), dim3(kRedBlock), 0, s, W, chi, zeta, rk, nd, nq, mu, kT,
                       partials);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(64), 0, s, partials, nblk, 1, out);
    return hipGetLastError();
}

hipError_t launch_density(const double *W, const double *chi, const double *zeta, const double *rk,
                          long long nd, int nq, double mu, const double *mu_dev, double kT, double h3,
                          double *rho, double *partials, int nblk, double *out, hipStream_t s) {
    hipLaunchKernelGGL(density_kernel, dim3(nblk), dim3(kRedBlock), 0, s, W, chi, zeta, rk, nd, nq, mu, mu_dev,
                       kT, h3, rho, partials);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(64), 0, s, partials, nblk, 3, out);
    return hipGetLastError();
}

hipError_t launch_brent_begin(BrentState *st, const BrentParams *prm, const double *ext, int nsnap, hipStream_t s) {
    hipLaunchKernelGGL(brent_begin_kernel, dim3((nsnap + 63) / 64), dim3(64), 0, s, st, prm, ext, nsnap);
    return hipGetLastError();
}

hipError_t launch_count_batch(const FermiSnap *fs, const BrentState *st, int nsnap, double *partials, int nblk,
                              hipStream_t s) {
    hipLaunchKernelGGL(count_batch_kernel, dim3(nblk, nsnap), dim3(kRedBlock), 0, s, fs, st, partials);
    return hipGetLastError();
}

hipError_t launch_brent_feed(BrentState *st, const double *partials, int nblk, int nsnap, hipStream_t s) {
    hipLaunchKernelGGL(brent_feed_kernel, dim3((nsnap + 63) / 64), dim3(64), 0, s, st, partials, nblk, nsnap);
    return hipGetLastError();
}

hipError_t static_scratch(double **ptr, size_t *bytes) {
    // The device address of `scratch` on the current device.  In host code the
    // array's name is not a device address; it is looked up once per device
    // (hipGetSymbolAddress with that device current) and cached.
    static std::mutex lock;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(lock);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *ptr = addr[dev];
    if (bytes) *bytes = sizeof(double) * kStaticScratchDoubles;
    return hipSuccess;
}

hipError_t launch_density_static(const double *mom, const double *ctab, const double *chi, const double *zeta,
                                 const double *rk, long long nd, int nq, double mu, double kT, double h3,
                                 double *rho, double *scratch_ptr, double **sums, hipStream_t s) {
    const int nblk = grid_for(nd, kRedBlock) < kStaticBlocks ? grid_for(nd, kRedBlock) : kStaticBlocks;
    double *partials = scratch_ptr;
    double *out = scratch_ptr + 3 * kStaticBlocks;
    hipLaunchKernelGGL(density_direct_kernel, dim3(nblk), dim3(kRedBlock), 0, s, mom, ctab, chi, zeta, rk, nd, nq,
                       mu, kT, h3, rho, partials);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(64), 0, s, partials, nblk, 3, out);
    *sums = out;
    return hipGetLastError();
}

#endif

}  // namespace sq
