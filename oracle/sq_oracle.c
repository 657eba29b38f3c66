/*
 * sq_oracle.c -- plain FP64 CPU oracle for the Clenshaw-Curtis spectral
 * quadrature (SQ) density/energy step of SQDFT (arXiv 1708.07913).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU path is checked against.  It shares no code with
 * the GPU library; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.
 *
 * Every routine follows the paper's statement of the method, in its order and
 * notation, with no blocking or fusion:
 *   grid, FD Laplacian weights, periodic index map, trapezoid rule  -- Sec. 3.1
 *   region of influence (cube of side 2 R_cut) and nodal Hamiltonian -- Sec. 3.1
 *   infinite-cell boundary semantics                                  -- Sec. 3 (intro)
 *   Lanczos spectral bounds, Chebyshev recurrence, moments,
 *   product property, coefficients, Fermi level (Brent), density      -- Sec. 3.2
 *   band-structure and entropy energies                               -- Sec. 3.3
 *   nonlocal atomic forces (recurrence to n_pl, FD gradient)         -- Sec. 3.4, 3.1
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - mesh refit h = L / round(L/h); cube half-width m = floor(R_cut/h + 1/2);
 *   - nodes at h*(i,j,k), flat index i + n (j + n k), cube index a + C (b + C c);
 *   - the Laplacian's d = 0 term counts f six times (diagonal 6 w_0);
 *   - stencil legs that leave the cube are dropped (zero Dirichlet at infinity);
 *     V_eff at a cube point is V_eff at its periodic image; every lattice image
 *     of a projector is a separate projector;
 *   - projector p = chi / N with h^3 sum p^2 = 1 over the full (unclipped)
 *     sphere |x - R| <= r_c (inclusive); its restriction to a cube is not
 *     renormalised;
 *   - product property with the corrected sign:
 *       rho^{2k} = 2 t_k.t_k - rho^0,  rho^{2k-1} = 2 t_k.t_{k-1} - rho^1;
 *   - recurrence stops at t^{n_pl/2} (n_pl/2 matrix-vector products);
 *   - coefficients by discrete orthogonality on N_q = n_pl + 1 Chebyshev-Gauss
 *     nodes, j = 0 halved;
 *   - Lanczos: fixed start vector v[a] = u(a) - 1/2, u(a) = (SplitMix64(a) >> 11)
 *     * 2^-53, normalised; Paige's ordering of the three-term recurrence without
 *     reorthogonalisation; k = min(n_lanczos, N_s) steps, earlier stop when
 *     beta_j <= 1e-13 * (Gershgorin bound of T_j); extreme eigenvalues of T_k by
 *     Sturm bisection to adjacent doubles; chi = (l_max + l_min)/2,
 *     zeta = (1 + margin)(l_max - l_min)/2;
 *   - Fermi level: Brent on N(mu) - N_e over
 *     [min(chi - zeta) - 40 sigma, max(chi + zeta) + 40 sigma].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define SQO_INFINITE_CELL 0
#define SQO_GAMMA 1

typedef struct {
    int i0, j0, k0;          /* lower corner of the sphere's bounding box (grid units) */
    int ni, nj, nk;          /* bounding box extent */
    int count;               /* number of grid points inside the sphere */
    int *ijk;                /* 3*count absolute grid coordinates on the infinite grid */
    double *p;               /* projector values p = chi / N */
    double gamma;
} sqo_atom;

typedef struct sqo {
    double L, h;
    int n, no, m, C;
    long nd, ns;
    int npl;
    double kT;
    int region;
    int n_lanczos;
    double margin;
    double w[7];             /* w[0..no] of the FD Laplacian */
    const double *veff;      /* n^3, borrowed */
    int natom;
    sqo_atom *atoms;
} sqo;

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: central finite-difference weights of order 2 n_o.              */
/*   w_0 = -(1/h^2) sum_{q=1}^{n_o} 1/q^2                                    */
/*   w_d = 2 (-1)^{d+1} / (h^2 d^2) * (n_o!)^2 / ((n_o-d)! (n_o+d)!)          */
/* ------------------------------------------------------------------------ */
static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= (double)i;
    return f;
}

int sqo_fd_weights(int fd_order, double h, double *w)
{
    if (fd_order < 2 || fd_order > 12 || (fd_order & 1)) return -1;
    int no = fd_order / 2;
    double s = 0.0;
    for (int q = 1; q <= no; q++) s += 1.0 / ((double)q * q);
    w[0] = -s / (h * h);
    for (int d = 1; d <= no; d++) {
        double sign = (d % 2 == 1) ? 1.0 : -1.0;
        double ratio = factorial(no) * factorial(no) / (factorial(no - d) * factorial(no + d));
        w[d] = 2.0 * sign / (h * h * (double)d * d) * ratio;
    }
    return 0;
}

/* SplitMix64 (S. Vigna): the first output of a generator seeded with `seed`. */
uint64_t sqo_splitmix64(uint64_t seed)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double sqo_unit(uint64_t a)
{
    return (double)(sqo_splitmix64(a) >> 11) * (1.0 / 9007199254740992.0);
}

static long imod(long a, long n)
{
    long r = a % n;
    return r < 0 ? r + n : r;
}

static long floordiv(long a, long b)
{
    long q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
    return q;
}

/* ------------------------------------------------------------------------ */
/* Nonlocal projectors: grid points of the infinite grid inside the sphere   */
/* |x - R| <= r_c, value chi(|x-R|) = exp(-|x-R|^2 / (2 s^2)), normalised so */
/* that h^3 sum p^2 = 1 (trapezoid rule, Sec. 3.1).                          */
/* ------------------------------------------------------------------------ */
static int build_atom(sqo_atom *A, const double *R, double sig, double rc, double gamma, double h)
{
    int lo[3], hi[3];
    for (int ax = 0; ax < 3; ax++) {
        lo[ax] = (int)ceil((R[ax] - rc) / h) - 1;
        hi[ax] = (int)floor((R[ax] + rc) / h) + 1;
    }
    A->i0 = lo[0]; A->j0 = lo[1]; A->k0 = lo[2];
    A->ni = hi[0] - lo[0] + 1; A->nj = hi[1] - lo[1] + 1; A->nk = hi[2] - lo[2] + 1;
    long cap = (long)A->ni * A->nj * A->nk;
    A->ijk = (int *)malloc(sizeof(int) * 3 * (cap > 0 ? cap : 1));
    A->p = (double *)malloc(sizeof(double) * (cap > 0 ? cap : 1));
    if (!A->ijk || !A->p) return -1;
    double rc2 = rc * rc;
    int cnt = 0;
    for (int k = lo[2]; k <= hi[2]; k++)
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                double dx = (double)i * h - R[0];
                double dy = (double)j * h - R[1];
                double dz = (double)k * h - R[2];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 <= rc2) {
                    A->ijk[3 * cnt + 0] = i;
                    A->ijk[3 * cnt + 1] = j;
                    A->ijk[3 * cnt + 2] = k;
                    A->p[cnt] = exp(-r2 / (2.0 * sig * sig));
                    cnt++;
                }
            }
    A->count = cnt;
    double s = 0.0;
    for (int e = 0; e < cnt; e++) s += A->p[e] * A->p[e];
    double norm = sqrt(h * h * h * s);
    for (int e = 0; e < cnt; e++) A->p[e] /= norm;
    A->gamma = gamma;
    return 0;
}

void sqo_destroy(sqo *S)
{
    if (!S) return;
    for (int a = 0; a < S->natom; a++) {
        free(S->atoms[a].ijk);
        free(S->atoms[a].p);
    }
    free(S->atoms);
    free(S);
}

sqo *sqo_create(double cell, double h_req, int fd_order, double rcut, int npl, double kT,
                int natom, const double *xyz, const double *kb, const double *veff,
                int region, int n_lanczos, double margin)
{
    if (cell <= 0 || h_req <= 0 || npl < 4 || (npl % 4) != 0 || npl > 1000 || kT <= 0) return NULL;
    if (n_lanczos < 1 || n_lanczos > 256 || margin < 0) return NULL;
    sqo *S = (sqo *)calloc(1, sizeof(sqo));
    if (!S) return NULL;
    S->L = cell;
    S->n = (int)floor(cell / h_req + 0.5);
    if (S->n < 1) { free(S); return NULL; }
    S->h = cell / S->n;
    if (sqo_fd_weights(fd_order, S->h, S->w) != 0) { free(S); return NULL; }
    S->no = fd_order / 2;
    S->m = (int)floor(rcut / S->h + 0.5);
    if (S->m < 1) { free(S); return NULL; }
    S->C = 2 * S->m + 1;
    S->nd = (long)S->n * S->n * S->n;
    S->region = region;
    S->ns = (region == SQO_GAMMA) ? S->nd : (long)S->C * S->C * S->C;
    S->npl = npl;
    S->kT = kT;
    S->n_lanczos = n_lanczos;
    S->margin = margin;
    S->veff = veff;
    S->natom = natom;
    S->atoms = (sqo_atom *)calloc(natom > 0 ? natom : 1, sizeof(sqo_atom));
    for (int a = 0; a < natom; a++) {
        if (build_atom(&S->atoms[a], xyz + 3 * a, kb[3 * a + 0], kb[3 * a + 1], kb[3 * a + 2], S->h) != 0) {
            sqo_destroy(S);
            return NULL;
        }
        if (region == SQO_GAMMA && 2.0 * kb[3 * a + 1] >= cell) {
            sqo_destroy(S);
            return NULL;
        }
    }
    return S;
}

int sqo_info(const sqo *S, int *n, int *m, long *nd, long *ns, double *h)
{
    *n = S->n; *m = S->m; *nd = S->nd; *ns = S->ns; *h = S->h;
    return 0;
}

int sqo_atom_table(const sqo *S, int a, int *count, const int **ijk, const double **p)
{
    if (a < 0 || a >= S->natom) return -1;
    *count = S->atoms[a].count;
    *ijk = S->atoms[a].ijk;
    *p = S->atoms[a].p;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Nodal Hamiltonian H_q (Sec. 3.1): restriction of the FD Hamiltonian       */
/* -1/2 nabla_h^2 + V_eff + V_nl to the region of influence of node q.       */
/* ------------------------------------------------------------------------ */

/* One projector image restricted to the region: (local index, value) pairs. */
typedef struct {
    int count;
    long *idx;
    double *p;
    double coef;             /* gamma * h^3 */
    int atom;                /* the atom this image belongs to */
} sqo_image;

typedef struct {
    long q;                  /* node */
    int qi, qj, qk;
    long *vidx;              /* periodic grid index of every local point */
    int nimg;
    sqo_image *img;
} sqo_region;

static void region_free(sqo_region *R)
{
    for (int i = 0; i < R->nimg; i++) {
        free(R->img[i].idx);
        free(R->img[i].p);
    }
    free(R->img);
    free(R->vidx);
}

static int region_add_image(sqo_region *R, int *cap, const sqo_image *im)
{
    if (R->nimg == *cap) {
        int nc = *cap ? 2 * *cap : 16;
        sqo_image *ni = (sqo_image *)realloc(R->img, sizeof(sqo_image) * nc);
        if (!ni) return -1;
        R->img = ni;
        *cap = nc;
    }
    R->img[R->nimg++] = *im;
    return 0;
}

/* Local index of infinite-grid point (i,j,k) in the cube of node q, or -1. */
static long cube_local(const sqo *S, const sqo_region *R, long i, long j, long k)
{
    long a = i - (R->qi - S->m), b = j - (R->qj - S->m), c = k - (R->qk - S->m);
    if (a < 0 || a >= S->C || b < 0 || b >= S->C || c < 0 || c >= S->C) return -1;
    return a + (long)S->C * (b + (long)S->C * c);
}

static int region_build(const sqo *S, long q, sqo_region *R)
{
    memset(R, 0, sizeof(*R));
    int n = S->n;
    R->q = q;
    R->qi = (int)(q % n);
    R->qj = (int)((q / n) % n);
    R->qk = (int)(q / ((long)n * n));
    double h3 = S->h * S->h * S->h;
    int cap = 0;
    R->vidx = (long *)malloc(sizeof(long) * S->ns);
    if (!R->vidx) return -1;
    if (S->region == SQO_GAMMA) {
        for (long g = 0; g < S->nd; g++) R->vidx[g] = g;
        for (int a = 0; a < S->natom; a++) {
            const sqo_atom *A = &S->atoms[a];
            sqo_image im;
            im.count = A->count;
            im.coef = A->gamma * h3;
            im.atom = a;
            im.idx = (long *)malloc(sizeof(long) * (A->count > 0 ? A->count : 1));
            im.p = (double *)malloc(sizeof(double) * (A->count > 0 ? A->count : 1));
            for (int e = 0; e < A->count; e++) {
                long i = imod(A->ijk[3 * e], n), j = imod(A->ijk[3 * e + 1], n), k = imod(A->ijk[3 * e + 2], n);
                im.idx[e] = i + (long)n * (j + (long)n * k);
                im.p[e] = A->p[e];
            }
            if (region_add_image(R, &cap, &im) != 0) return -1;
        }
        return 0;
    }
    int C = S->C, m = S->m;
    for (int c = 0; c < C; c++)
        for (int b = 0; b < C; b++)
            for (int a = 0; a < C; a++) {
                long i = imod(R->qi - m + a, n), j = imod(R->qj - m + b, n), k = imod(R->qk - m + c, n);
                R->vidx[a + (long)C * (b + (long)C * c)] = i + (long)n * (j + (long)n * k);
            }
    /* every lattice image (atom a, translation t) whose sphere meets the cube */
    for (int a = 0; a < S->natom; a++) {
        const sqo_atom *A = &S->atoms[a];
        long lo[3] = {A->i0, A->j0, A->k0};
        long ext[3] = {A->ni, A->nj, A->nk};
        long qc[3] = {R->qi, R->qj, R->qk};
        long tlo[3], thi[3];
        for (int ax = 0; ax < 3; ax++) {
            /* box [lo + n t, lo + ext - 1 + n t] meets [qc - m, qc + m] */
            tlo[ax] = floordiv(qc[ax] - m - (lo[ax] + ext[ax] - 1) + n - 1, n);
            thi[ax] = floordiv(qc[ax] + m - lo[ax], n);
        }
        for (long tz = tlo[2]; tz <= thi[2]; tz++)
            for (long ty = tlo[1]; ty <= thi[1]; ty++)
                for (long tx = tlo[0]; tx <= thi[0]; tx++) {
                    int cnt = 0;
                    for (int e = 0; e < A->count; e++)
                        if (cube_local(S, R, A->ijk[3 * e] + n * tx, A->ijk[3 * e + 1] + n * ty,
                                       A->ijk[3 * e + 2] + n * tz) >= 0)
                            cnt++;
                    if (cnt == 0) continue;
                    sqo_image im;
                    im.count = cnt;
                    im.coef = A->gamma * h3;
                    im.atom = a;
                    im.idx = (long *)malloc(sizeof(long) * cnt);
                    im.p = (double *)malloc(sizeof(double) * cnt);
                    cnt = 0;
                    for (int e = 0; e < A->count; e++) {
                        long l = cube_local(S, R, A->ijk[3 * e] + n * tx, A->ijk[3 * e + 1] + n * ty,
                                            A->ijk[3 * e + 2] + n * tz);
                        if (l >= 0) {
                            im.idx[cnt] = l;
                            im.p[cnt] = A->p[e];
                            cnt++;
                        }
                    }
                    if (region_add_image(R, &cap, &im) != 0) return -1;
                }
    }
    return 0;
}

/* y = H_q x (unscaled nodal Hamiltonian). */
static void apply_h(const sqo *S, const sqo_region *R, const double *x, double *y)
{
    int no = S->no;
    if (S->region == SQO_GAMMA) {
        long n = S->n;
        for (long k = 0; k < n; k++)
            for (long j = 0; j < n; j++)
                for (long i = 0; i < n; i++) {
                    long g = i + n * (j + n * k);
                    double lap = 6.0 * S->w[0] * x[g];
                    for (int d = 1; d <= no; d++) {
                        lap += S->w[d] * (x[imod(i + d, n) + n * (j + n * k)] + x[imod(i - d, n) + n * (j + n * k)]);
                        lap += S->w[d] * (x[i + n * (imod(j + d, n) + n * k)] + x[i + n * (imod(j - d, n) + n * k)]);
                        lap += S->w[d] * (x[i + n * (j + n * imod(k + d, n))] + x[i + n * (j + n * imod(k - d, n))]);
                    }
                    y[g] = -0.5 * lap + S->veff[g] * x[g];
                }
    } else {
        long C = S->C;
        for (long c = 0; c < C; c++)
            for (long b = 0; b < C; b++)
                for (long a = 0; a < C; a++) {
                    long l = a + C * (b + C * c);
                    double lap = 6.0 * S->w[0] * x[l];
                    for (int d = 1; d <= no; d++) {
                        if (a + d < C) lap += S->w[d] * x[l + d];
                        if (a - d >= 0) lap += S->w[d] * x[l - d];
                        if (b + d < C) lap += S->w[d] * x[l + d * C];
                        if (b - d >= 0) lap += S->w[d] * x[l - d * C];
                        if (c + d < C) lap += S->w[d] * x[l + d * C * C];
                        if (c - d >= 0) lap += S->w[d] * x[l - d * C * C];
                    }
                    y[l] = -0.5 * lap + S->veff[R->vidx[l]] * x[l];
                }
    }
    for (int I = 0; I < R->nimg; I++) {
        const sqo_image *im = &R->img[I];
        double s = 0.0;
        for (int e = 0; e < im->count; e++) s += im->p[e] * x[im->idx[e]];
        for (int e = 0; e < im->count; e++) y[im->idx[e]] += im->coef * s * im->p[e];
    }
}

static long center_index(const sqo *S, long q)
{
    if (S->region == SQO_GAMMA) return q;
    long C = S->C, m = S->m;
    return m + C * (m + C * m);
}

int sqo_matvec(const sqo *S, long q, const double *x, double *y)
{
    if (q < 0 || q >= S->nd) return -1;
    sqo_region R;
    if (region_build(S, q, &R) != 0) { region_free(&R); return -2; }
    apply_h(S, &R, x, y);
    region_free(&R);
    return 0;
}

int sqo_region_images(const sqo *S, long q)
{
    sqo_region R;
    if (region_build(S, q, &R) != 0) { region_free(&R); return -1; }
    int k = R.nimg;
    region_free(&R);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Spectral bounds (Sec. 3.2): Lanczos on H_q, extremes of the tridiagonal   */
/* by Sturm bisection.                                                       */
/* ------------------------------------------------------------------------ */

/* Number of eigenvalues of the symmetric tridiagonal (a, b) below x. */
static int sturm_count(int k, const double *a, const double *b, double x, double pivmin)
{
    int cnt = 0;
    double d = a[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0) cnt++;
    for (int i = 1; i < k; i++) {
        d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        if (d < 0) cnt++;
    }
    return cnt;
}

/* Smallest x (to adjacent doubles) with at least `target` eigenvalues below x. */
static double sturm_bisect(int k, const double *a, const double *b, int target)
{
    double lo = INFINITY, hi = -INFINITY, bmax2 = 0.0;
    for (int i = 0; i < k; i++) {
        double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < k - 1 ? fabs(b[i]) : 0.0);
        if (a[i] - r < lo) lo = a[i] - r;
        if (a[i] + r > hi) hi = a[i] + r;
        if (i < k - 1 && b[i] * b[i] > bmax2) bmax2 = b[i] * b[i];
    }
    double pivmin = DBL_MIN * (bmax2 > 1.0 ? bmax2 : 1.0);
    for (int it = 0; it < 256; it++) {
        double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(k, a, b, mid, pivmin) >= target) hi = mid;
        else lo = mid;
    }
    return hi;
}

int sqo_tridiag_extremes(int k, const double *a, const double *b, double *lmin, double *lmax)
{
    if (k < 1) return -1;
    *lmin = sturm_bisect(k, a, b, 1);
    *lmax = sturm_bisect(k, a, b, k);
    return 0;
}

static double dot(long n, const double *x, const double *y)
{
    double s = 0.0;
    for (long i = 0; i < n; i++) s += x[i] * y[i];
    return s;
}

/* Lanczos for one node; returns the number of steps k and alpha/beta. */
static int lanczos_node(const sqo *S, const sqo_region *R, double *alpha, double *beta,
                        double *v, double *vprev, double *w)
{
    long ns = S->ns;
    int kmax = S->n_lanczos;
    if ((long)kmax > ns) kmax = (int)ns;
    for (long a = 0; a < ns; a++) v[a] = sqo_unit((uint64_t)a) - 0.5;
    double nrm = sqrt(dot(ns, v, v));
    for (long a = 0; a < ns; a++) v[a] /= nrm;
    for (long a = 0; a < ns; a++) vprev[a] = 0.0;
    double bprev = 0.0, gersh = 0.0;
    int k = kmax;
    for (int j = 0; j < kmax; j++) {
        apply_h(S, R, v, w);
        for (long a = 0; a < ns; a++) w[a] -= bprev * vprev[a];
        double al = dot(ns, w, v);
        for (long a = 0; a < ns; a++) w[a] -= al * v[a];
        double be = sqrt(dot(ns, w, w));
        alpha[j] = al;
        beta[j] = be;
        double g = fabs(al) + be + bprev;
        if (g > gersh) gersh = g;
        if (j == kmax - 1 || be <= 1e-13 * gersh) { k = j + 1; break; }
        for (long a = 0; a < ns; a++) {
            vprev[a] = v[a];
            v[a] = w[a] / be;
        }
        bprev = be;
    }
    return k;
}

int sqo_lanczos(const sqo *S, long q, double *alpha, double *beta, int *k)
{
    if (q < 0 || q >= S->nd) return -1;
    sqo_region R;
    if (region_build(S, q, &R) != 0) { region_free(&R); return -2; }
    double *buf = (double *)malloc(sizeof(double) * 3 * S->ns);
    *k = lanczos_node(S, &R, alpha, beta, buf, buf + S->ns, buf + 2 * S->ns);
    free(buf);
    region_free(&R);
    return 0;
}

int sqo_bounds(const sqo *S, const long *nodes, long count, double *lmin, double *lmax, int *steps)
{
    int err = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 3 * S->ns);
        double al[256], be[256];
#pragma omp for schedule(dynamic, 4)
        for (long t = 0; t < count; t++) {
            long q = nodes ? nodes[t] : t;
            sqo_region R;
            if (!buf || region_build(S, q, &R) != 0) {
#pragma omp atomic write
                err = -2;
                continue;
            }
            int k = lanczos_node(S, &R, al, be, buf, buf + S->ns, buf + 2 * S->ns);
            sqo_tridiag_extremes(k, al, be, &lmin[t], &lmax[t]);
            if (steps) steps[t] = k;
            region_free(&R);
        }
        free(buf);
    }
    return err;
}

static void scale_bounds(const sqo *S, double lmin, double lmax, double *chi, double *zeta)
{
    *chi = 0.5 * (lmax + lmin);
    *zeta = (1.0 + S->margin) * 0.5 * (lmax - lmin);
}

/* ------------------------------------------------------------------------ */
/* Chebyshev recurrence and moments (Sec. 3.2).                              */
/*   t^0 = e_q, t^1 = Hhat t^0, t^{k+1} = 2 Hhat t^k - t^{k-1},               */
/*   Hhat = (H_q - chi I) / zeta                                             */
/*   rho^j = t^j[q] for j <= n_pl/2, higher moments by the product property. */
/* ------------------------------------------------------------------------ */
static void apply_hhat(const sqo *S, const sqo_region *R, double chi, double zeta,
                       const double *x, double *y)
{
    apply_h(S, R, x, y);
    for (long a = 0; a < S->ns; a++) y[a] = (y[a] - chi * x[a]) / zeta;
}

int sqo_moments(const sqo *S, const long *nodes, long count, const double *lmin, const double *lmax,
                double *mom)
{
    int npl = S->npl, half = npl / 2;
    int err = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 4 * S->ns);
#pragma omp for schedule(dynamic, 4)
        for (long t = 0; t < count; t++) {
            long q = nodes ? nodes[t] : t;
            sqo_region R;
            if (!buf || region_build(S, q, &R) != 0) {
#pragma omp atomic write
                err = -2;
                continue;
            }
            double chi, zeta;
            scale_bounds(S, lmin[t], lmax[t], &chi, &zeta);
            double *tm1 = buf, *t0 = buf + S->ns, *tp1 = buf + 2 * S->ns, *hv = buf + 3 * S->ns;
            double *row = mom + t * (long)(npl + 1);
            long c = center_index(S, q);
            for (long a = 0; a < S->ns; a++) tm1[a] = 0.0;
            tm1[c] = 1.0;                                /* t^0 = w_q = e_q */
            apply_hhat(S, &R, chi, zeta, tm1, t0);      /* t^1 = Hhat w_q  */
            row[0] = tm1[c];
            row[1] = t0[c];
            /* t^{k-1} = tm1, t^k = t0 */
            for (int k = 1; k <= half; k++) {
                if (k > half / 2) {
                    row[2 * k] = 2.0 * dot(S->ns, t0, t0) - row[0];
                    row[2 * k - 1] = 2.0 * dot(S->ns, t0, tm1) - row[1];
                }
                if (k == half) break;
                apply_hhat(S, &R, chi, zeta, t0, hv);
                for (long a = 0; a < S->ns; a++) tp1[a] = 2.0 * hv[a] - tm1[a];
                row[k + 1] = tp1[c];
                double *tmp = tm1; tm1 = t0; t0 = tp1; tp1 = tmp;
            }
            region_free(&R);
        }
        free(buf);
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev coefficients by discrete orthogonality (Sec. 3.2, 3.3).         */
/* c^j, d^j, e^j of g(r), r g(r), s(g(r)) with                               */
/*   g(r) = 1 / (1 + exp((zeta r + chi - mu) / sigma)),                      */
/*   s(g) = g log g + (1 - g) log(1 - g);  j = 0 halved.                     */
/* ------------------------------------------------------------------------ */
static double fermi(double x)
{
    return 1.0 / (1.0 + exp(x));
}

/* g log g + (1-g) log(1-g) at g = fermi(x), written so that 0 log 0 = 0. */
static double entropy_fn(double x)
{
    double ax = fabs(x), e = exp(-ax);
    return -(log1p(e) + ax * e / (1.0 + e));
}

int sqo_coefficients(const sqo *S, double mu, double lmin, double lmax, double *c, double *d, double *e)
{
    int npl = S->npl, Nq = npl + 1;
    double chi, zeta;
    scale_bounds(S, lmin, lmax, &chi, &zeta);
    for (int j = 0; j <= npl; j++) {
        double sc = 0.0, sd = 0.0, se = 0.0;
        for (int k = 0; k < Nq; k++) {
            double th = M_PI * (k + 0.5) / Nq;
            double r = cos(th);
            double x = (zeta * r + chi - mu) / S->kT;
            double g = fermi(x);
            double cj = cos(j * th);
            sc += g * cj;
            sd += r * g * cj;
            se += entropy_fn(x) * cj;
        }
        double f = (j == 0 ? 1.0 : 2.0) / Nq;
        if (c) c[j] = f * sc;
        if (d) d[j] = f * sd;
        if (e) e[j] = f * se;
    }
    return 0;
}

/* N(mu) = 2 sum_q sum_j c_q^j rho_q^j over the given nodes. */
double sqo_electron_count(const sqo *S, long count, const double *lmin, const double *lmax,
                          const double *mom, double mu)
{
    int npl = S->npl;
    double *per = (double *)malloc(sizeof(double) * (count > 0 ? count : 1));
#pragma omp parallel
    {
        double c[1024];
#pragma omp for schedule(static)
        for (long t = 0; t < count; t++) {
            sqo_coefficients(S, mu, lmin[t], lmax[t], c, NULL, NULL);
            double s = 0.0;
            for (int j = 0; j <= npl; j++) s += c[j] * mom[t * (long)(npl + 1) + j];
            per[t] = s;
        }
    }
    long double tot = 0.0L;
    for (long t = 0; t < count; t++) tot += per[t];
    free(per);
    return 2.0 * (double)tot;
}

/* Brent's root finder (inverse quadratic interpolation / secant / bisection)
 * on f(mu) = N(mu) - N_e over the spectral bracket. */
int sqo_fermi_level(const sqo *S, long count, const double *lmin, const double *lmax,
                    const double *mom, double ne, double xtol, double frtol, int maxit,
                    double *mu_out, int *iters)
{
    double lo = INFINITY, hi = -INFINITY;
    for (long t = 0; t < count; t++) {
        double chi, zeta;
        scale_bounds(S, lmin[t], lmax[t], &chi, &zeta);
        if (chi - zeta < lo) lo = chi - zeta;
        if (chi + zeta > hi) hi = chi + zeta;
    }
    lo -= 40.0 * S->kT;
    hi += 40.0 * S->kT;
    double ftol = frtol * ne;
    double a = lo, b = hi;
    double fa = sqo_electron_count(S, count, lmin, lmax, mom, a) - ne;
    double fb = sqo_electron_count(S, count, lmin, lmax, mom, b) - ne;
    if ((fa > 0 && fb > 0) || (fa < 0 && fb < 0)) return -3;
    double c = a, fc = fa, dstep = b - a, estep = dstep;
    for (int it = 1; it <= maxit; it++) {
        if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) {
            c = a; fc = fa; dstep = b - a; estep = dstep;
        }
        if (fabs(fc) < fabs(fb)) {
            a = b; b = c; c = a;
            fa = fb; fb = fc; fc = fa;
        }
        double tol1 = 2.0 * DBL_EPSILON * fabs(b) + 0.5 * xtol;
        double xm = 0.5 * (c - b);
        if (fabs(xm) <= tol1 || fabs(fb) <= ftol) {
            *mu_out = b;
            if (iters) *iters = it;
            return 0;
        }
        if (fabs(estep) >= tol1 && fabs(fa) > fabs(fb)) {
            double s = fb / fa, p, qq;
            if (a == c) {
                p = 2.0 * xm * s;
                qq = 1.0 - s;
            } else {
                double qa = fa / fc, r = fb / fc;
                p = s * (2.0 * xm * qa * (qa - r) - (b - a) * (r - 1.0));
                qq = (qa - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) qq = -qq;
            p = fabs(p);
            double min1 = 3.0 * xm * qq - fabs(tol1 * qq);
            double min2 = fabs(estep * qq);
            if (2.0 * p < (min1 < min2 ? min1 : min2)) {
                estep = dstep;
                dstep = p / qq;
            } else {
                dstep = xm;
                estep = dstep;
            }
        } else {
            dstep = xm;
            estep = dstep;
        }
        a = b;
        fa = fb;
        if (fabs(dstep) > tol1) b += dstep;
        else b += (xm >= 0 ? tol1 : -tol1);
        fb = sqo_electron_count(S, count, lmin, lmax, mom, b) - ne;
    }
    return -5;
}

/* rho_q = (2/h^3) sum_j c^j rho^j; E_band = 2 sum (chi c + zeta d) rho^j;
 * E_ent = 2 sigma sum e rho^j.  out = {E_band, E_ent, E_band + E_ent, h^3 sum rho}. */
int sqo_density_energy(const sqo *S, long count, const double *lmin, const double *lmax,
                       const double *mom, double mu, double *rho, double *out)
{
    int npl = S->npl;
    double h3 = S->h * S->h * S->h;
    double *eb = (double *)malloc(sizeof(double) * (count > 0 ? count : 1));
    double *en = (double *)malloc(sizeof(double) * (count > 0 ? count : 1));
#pragma omp parallel
    {
        double c[1024], d[1024], e[1024];
#pragma omp for schedule(static)
        for (long t = 0; t < count; t++) {
            double chi, zeta;
            scale_bounds(S, lmin[t], lmax[t], &chi, &zeta);
            sqo_coefficients(S, mu, lmin[t], lmax[t], c, d, e);
            const double *r = mom + t * (long)(npl + 1);
            double sr = 0.0, sb = 0.0, se = 0.0;
            for (int j = 0; j <= npl; j++) {
                sr += c[j] * r[j];
                sb += (chi * c[j] + zeta * d[j]) * r[j];
                se += e[j] * r[j];
            }
            rho[t] = 2.0 / h3 * sr;
            eb[t] = 2.0 * sb;
            en[t] = 2.0 * S->kT * se;
        }
    }
    long double tb = 0.0L, te = 0.0L, tr = 0.0L;
    for (long t = 0; t < count; t++) {
        tb += eb[t];
        te += en[t];
        tr += rho[t];
    }
    out[0] = (double)tb;
    out[1] = (double)te;
    out[2] = (double)(tb + te);
    out[3] = h3 * (double)tr;
    free(eb);
    free(en);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Nonlocal atomic forces (Sec. 3.4, nonlocal component).                    */
/*   f_I = -4 sum_{I' images of I} sum_q w_q^T V_q^{I'} grad_{h,q} u_q,       */
/*   u_q = sum_{j=0}^{n_pl} c_q^j t_q^j  (the recurrence run to n_pl),        */
/* with V^{I'} = gamma h^3 p p^T, so w_q^T V^{I'} = gamma h^3 p(q) p^T, and   */
/* grad_{h,q} the central-difference gradient of Sec. 3.1 restricted to the  */
/* region of influence (legs leaving the cube dropped; periodic in the       */
/* whole-cell mode).  Only nodes inside some projector sphere contribute.    */
/* ------------------------------------------------------------------------ */
static void fd_gradient_weights(int no, double h, double *wt)
{
    double f2 = factorial(no) * factorial(no);
    wt[0] = 0.0;
    for (int d = 1; d <= no; d++)
        wt[d] = ((d % 2) ? 1.0 : -1.0) / (h * d) * f2 / (factorial(no - d) * factorial(no + d));
}

/* (grad_{h,q} u)(l) along axis ax for local point l of the region. */
static double grad_at(const sqo *S, const double *wt, const double *u, long l, int ax)
{
    double g = 0.0;
    if (S->region == SQO_GAMMA) {
        long n = S->n, i = l % n, j = (l / n) % n, k = l / (n * n);
        for (int d = 1; d <= S->no; d++) {
            long ip = i, jp = j, kp = k, im = i, jm = j, km = k;
            if (ax == 0) { ip = imod(i + d, n); im = imod(i - d, n); }
            if (ax == 1) { jp = imod(j + d, n); jm = imod(j - d, n); }
            if (ax == 2) { kp = imod(k + d, n); km = imod(k - d, n); }
            g += wt[d] * (u[ip + n * (jp + n * kp)] - u[im + n * (jm + n * km)]);
        }
        return g;
    }
    long C = S->C, a = l % C, b = (l / C) % C, c = l / (C * C);
    long pos = ax == 0 ? a : (ax == 1 ? b : c);
    long stride = ax == 0 ? 1 : (ax == 1 ? C : C * C);
    for (int d = 1; d <= S->no; d++) {
        if (pos + d < C) g += wt[d] * u[l + d * stride];
        if (pos - d >= 0) g -= wt[d] * u[l - d * stride];
    }
    return g;
}

#define SQO_MAX_CENTRE_IMAGES 16

int sqo_nl_forces(const sqo *S, const long *nodes, long count, const double *lmin, const double *lmax,
                  double mu, double *forces)
{
    int npl = S->npl;
    int err = 0;
    double wt[8];
    fd_gradient_weights(S->no, S->h, wt);
    /* per node: up to SQO_MAX_CENTRE_IMAGES (atom, force) contributions, summed
       afterwards in node order */
    int *atom = (int *)malloc(sizeof(int) * SQO_MAX_CENTRE_IMAGES * (count > 0 ? count : 1));
    double *fc = (double *)malloc(sizeof(double) * 3 * SQO_MAX_CENTRE_IMAGES * (count > 0 ? count : 1));
    if (!atom || !fc) { free(atom); free(fc); return -2; }
    for (long t = 0; t < SQO_MAX_CENTRE_IMAGES * count; t++) atom[t] = -1;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 5 * S->ns);
        double *c = (double *)malloc(sizeof(double) * (npl + 1));
#pragma omp for schedule(dynamic, 4)
        for (long t = 0; t < count; t++) {
            long q = nodes ? nodes[t] : t;
            sqo_region R;
            if (!buf || !c || region_build(S, q, &R) != 0) {
#pragma omp atomic write
                err = -2;
                continue;
            }
            long lc = center_index(S, q);
            /* images whose sphere contains the node, with p(q) */
            int ci[SQO_MAX_CENTRE_IMAGES];
            double pc[SQO_MAX_CENTRE_IMAGES];
            int nc = 0;
            for (int I = 0; I < R.nimg; I++)
                for (int e = 0; e < R.img[I].count; e++)
                    if (R.img[I].idx[e] == lc && nc < SQO_MAX_CENTRE_IMAGES) {
                        ci[nc] = I;
                        pc[nc] = R.img[I].p[e];
                        nc++;
                    }
            if (nc == 0) { region_free(&R); continue; }
            double chi, zeta;
            scale_bounds(S, lmin[t], lmax[t], &chi, &zeta);
            sqo_coefficients(S, mu, lmin[t], lmax[t], c, NULL, NULL);
            double *tm1 = buf, *t0 = buf + S->ns, *tp1 = buf + 2 * S->ns, *hv = buf + 3 * S->ns;
            double *u = buf + 4 * S->ns;
            for (long a = 0; a < S->ns; a++) tm1[a] = 0.0;
            tm1[lc] = 1.0;                               /* t^0 = w_q */
            apply_hhat(S, &R, chi, zeta, tm1, t0);      /* t^1 = Hhat w_q */
            for (long a = 0; a < S->ns; a++) u[a] = c[0] * tm1[a] + c[1] * t0[a];
            for (int k = 1; k < npl; k++) {             /* t^{k+1}, k + 1 = 2 .. n_pl */
                apply_hhat(S, &R, chi, zeta, t0, hv);
                for (long a = 0; a < S->ns; a++) tp1[a] = 2.0 * hv[a] - tm1[a];
                for (long a = 0; a < S->ns; a++) u[a] += c[k + 1] * tp1[a];
                double *tmp = tm1; tm1 = t0; t0 = tp1; tp1 = tmp;
            }
            for (int m = 0; m < nc; m++) {
                const sqo_image *im = &R.img[ci[m]];
                double sv[3] = {0.0, 0.0, 0.0};        /* p^T grad_{h,q} u */
                for (int e = 0; e < im->count; e++)
                    for (int ax = 0; ax < 3; ax++) sv[ax] += im->p[e] * grad_at(S, wt, u, im->idx[e], ax);
                atom[t * SQO_MAX_CENTRE_IMAGES + m] = im->atom;
                for (int ax = 0; ax < 3; ax++)
                    fc[(t * SQO_MAX_CENTRE_IMAGES + m) * 3 + ax] = -4.0 * im->coef * pc[m] * sv[ax];
            }
            region_free(&R);
        }
        free(buf);
        free(c);
    }
    for (long a = 0; a < 3L * S->natom; a++) forces[a] = 0.0;
    for (long t = 0; t < count; t++)
        for (int m = 0; m < SQO_MAX_CENTRE_IMAGES; m++) {
            int at = atom[t * SQO_MAX_CENTRE_IMAGES + m];
            if (at < 0) continue;
            for (int ax = 0; ax < 3; ax++) forces[3 * at + ax] += fc[(t * SQO_MAX_CENTRE_IMAGES + m) * 3 + ax];
        }
    free(atom);
    free(fc);
    return err;
}

int sqo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
