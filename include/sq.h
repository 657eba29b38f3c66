/*
 * sq.h -- C ABI of libsq: the spectral-quadrature (SQ) density/energy step of
 * SQDFT (arXiv 1708.07913) on one AMD MI355X (gfx950) GPU.
 *
 * The library computes, for every node q of a periodic finite-difference grid,
 * the Clenshaw-Curtis SQ electron density and energies of the infinite crystal
 * whose unit cell is the cubic domain (Sec. 3, infinite-cell SQ):
 *
 *   bounds    l_min, l_max of the nodal Hamiltonian H_q by Lanczos  (Sec. 3.2)
 *   moments   rho_q^j = e_q^T T_j(Hhat_q) e_q, j = 0..n_pl           (Sec. 3.2,
 *             Chebyshev three-term recurrence + product property)
 *   Fermi     mu with 2 sum_q sum_j c_q^j(mu) rho_q^j = N_e (Brent)  (Sec. 3.2)
 *   density   rho_q = (2/h^3) sum_j c_q^j rho_q^j                    (Sec. 3.2)
 *   energies  E_band = 2 sum (chi c + zeta d) rho^j,
 *             E_ent  = 2 sigma sum e rho^j                           (Sec. 3.3)
 *
 * H_q is the restriction to the cube of side 2 R_cut around q (the region of
 * influence, Sec. 3.1) of H = -1/2 lap_h + V_eff + sum_I gamma_I h^3 p_I p_I^T:
 * central FD Laplacian of order fd_order (Sec. 3.1), V_eff sampled at the
 * periodic image of each cube point, one s-type Kleinman-Bylander projector per
 * atom image (every lattice image is a separate projector), stencil legs that
 * leave the cube dropped (zero Dirichlet at infinity).
 *
 * Units: lengths in Bohr, energies and kT in Hartree.
 * Grid: n = round(cell / h) nodes per axis, h_eff = cell / n, node (i,j,k) at
 * h_eff (i,j,k), flat index i + n (j + n k).  Cube half-width
 * m = floor(R_cut / h_eff + 1/2), N_s = (2m+1)^3.
 *
 * Memory: every device buffer is owned by the caller (e.g. allocated through
 * PyTorch) and borrowed by the library for the duration of a call; the
 * library never allocates or frees device memory.  Pointers marked (device)
 * must be device pointers on the current HIP device; pointers marked (host)
 * are ordinary host memory.
 *
 * Streams: every call takes the caller's hipStream_t as `void *stream` (NULL
 * = the null stream) and enqueues its kernels there.  Calls that return host
 * scalars (or report device-side errors) synchronise that stream before
 * returning.
 *
 * Errors: every call returns an sq_status; no C++ exception crosses the ABI.
 * On failure sq_last_error() returns a message for the calling thread.
 *
 * Call order per V_eff: sq_setup -> sq_query -> sq_bind -> (sq_spectral_bounds
 * | sq_set_bounds) -> sq_moments -> sq_fermi_level -> sq_density_energy.
 * Out-of-order calls return SQ_ESTATE.  sq_update_veff invalidates bounds.
 */
#ifndef SQ_H
#define SQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sq_ctx sq_ctx;

typedef enum {
    SQ_OK = 0,
    SQ_EINVAL = -1,      /* invalid argument */
    SQ_ENOMEM = -2,      /* workspace too small / host allocation failed */
    SQ_EDEVICE = -3,     /* HIP runtime error or kernel fault */
    SQ_ESTATE = -4,      /* call out of order */
    SQ_ENOCONV = -5,     /* Fermi-level search did not converge / no bracket */
    SQ_EBOUNDS = -6,     /* a moment left [-1, 1]: spectral bounds too tight */
    SQ_ECAPACITY = -7    /* a per-node table exceeded its compiled capacity */
} sq_status;

enum { SQ_FP64 = 0, SQ_FP32_MIXED = 1 };

typedef struct sq_options {
    /* SQ_FP64: everything in FP64.  SQ_FP32_MIXED: recurrence vectors, potential
     * window and stencil pair sums in FP32, every accumulation (stencil sum,
     * projector dots, moments), the Lanczos bounds, coefficients, Fermi solve
     * and energies in FP64. */
    int precision;
    int n_lanczos;       /* Lanczos steps per node, 1..256 (default 50) */
    double margin;       /* zeta = (1 + margin)(l_max - l_min)/2 (default 0.05) */
    double mu_xtol;      /* Brent stop: bracket half-width (Ha), default 1e-14 */
    double ne_rtol;      /* Brent stop: |N(mu) - N_e| <= ne_rtol * N_e, default 1e-13 */
    int max_brent;       /* Brent iteration cap (default 200) */
    int workgroups;      /* persistent workgroups for the recurrence kernels (0 = auto) */
} sq_options;

/* Fill *opt with the defaults above. */
void sq_default_options(sq_options *opt);

/*
 * Create a context for one snapshot (Sec. 3.1 problem statement).
 *   cell      cubic cell edge L (> 0)
 *   h         requested mesh size (> 0); refitted to L / round(L / h)
 *   fd_order  even order 2 n_o of the central FD Laplacian, 2..12
 *   rcut      R_cut: half-side of the cubic region of influence; 1 <= m <= 18
 *             (cube side 2m + 1 <= 37; SQ_EINVAL beyond)
 *   npl       quadrature order n_pl, a multiple of 4 in [4, 1000]
 *   kT        smearing sigma (Ha, > 0)
 *   natom     number of atoms (>= 0)
 *   atom_xyz  (host) natom x 3 Cartesian positions, any real values (images
 *             are taken care of)
 *   kb        (host) natom x 3: projector Gaussian width s, cut radius r_c and
 *             energy gamma; chi(r) = exp(-r^2/(2 s^2)) for r <= r_c, normalised
 *             so that h^3 sum chi^2 = 1 over the full sphere; may be NULL only
 *             if natom == 0
 *   opt       (host) options or NULL for the defaults
 * Host inputs are copied.  On success *ctx owns host tables only.
 * SQ_ECAPACITY if more than four projector spheres overlap at a grid point
 * (more than two for cubes wider than 31 points).
 */
int sq_setup(sq_ctx **ctx, double cell, double h, int fd_order, double rcut, int npl,
             double kT, int natom, const double *atom_xyz, const double *kb,
             const sq_options *opt);

/* Sizes of a context: grid points per axis n, cube half-width m, node count
 * n^3 and the device workspace (bytes) that sq_bind needs.  Any out pointer
 * may be NULL. */
int sq_query(const sq_ctx *ctx, int *n, int *m, long long *n_nodes, size_t *workspace_bytes);

/* Bind a caller-allocated device workspace (>= workspace_bytes, 256-byte
 * aligned) and the effective potential veff (device, n^3 FP64, flat index
 * i + n (j + n k)); uploads the projector tables.  veff is borrowed until the
 * next sq_bind / sq_update_veff or sq_destroy.  Synchronises `stream`. */
int sq_bind(sq_ctx *ctx, void *workspace, size_t bytes, const double *veff, void *stream);

/* Replace V_eff (device, n^3 FP64) for the next SCF iteration; bounds must be
 * recomputed or re-injected afterwards. */
int sq_update_veff(sq_ctx *ctx, const double *veff, void *stream);

/* Spectral bounds of every H_q by n_lanczos Lanczos steps (Sec. 3.2): writes
 * l_min, l_max (device, N_d FP64 each; either may be NULL) and keeps
 * chi_q = (l_max + l_min)/2, zeta_q = (1 + margin)(l_max - l_min)/2 in the
 * workspace.  Synchronises `stream`. */
int sq_spectral_bounds(sq_ctx *ctx, double *lmin, double *lmax, void *stream);

/* Inject bounds instead of computing them (device, N_d FP64 each): the same
 * chi/zeta rule is applied.  Used to compare two implementations of the
 * recurrence on identical bounds. */
int sq_set_bounds(sq_ctx *ctx, const double *lmin, const double *lmax, void *stream);

/* Chebyshev moments (Sec. 3.2): moments (device, N_d x (n_pl + 1) FP64,
 * row-major by node) receives rho_q^j = e_q^T T_j(Hhat_q) e_q.  Columns
 * 0..n_pl/2 come from the recurrence t^{k+1} = 2 Hhat t^k - t^{k-1},
 * columns above from rho^{2k} = 2 t^k.t^k - rho^0 and
 * rho^{2k-1} = 2 t^k.t^{k-1} - rho^1.  Returns SQ_EBOUNDS if a moment leaves
 * [-1, 1] by more than rounding.  Synchronises `stream`. */
int sq_moments(sq_ctx *ctx, double *moments, void *stream);

/* Fermi level (Sec. 3.2): Brent's method on N(mu) - N_e over
 * [min_q(chi - zeta) - 40 kT, max_q(chi + zeta) + 40 kT], with the Chebyshev
 * coefficients taken by discrete orthogonality on n_pl + 1 Chebyshev-Gauss
 * nodes.  moments (device) as written by sq_moments; *mu (host) receives the
 * result.  0 < n_electrons < 2 N_d.  Synchronises `stream`. */
int sq_fermi_level(sq_ctx *ctx, const double *moments, double n_electrons, double *mu,
                   void *stream);

/* Density and energies at Fermi level mu (Sec. 3.2-3.3): rho (device, N_d
 * FP64) and energies (host, 4 FP64) = {E_band, E_ent, E_band + E_ent,
 * h^3 sum_q rho_q}.  Synchronises `stream`. */
int sq_density_energy(sq_ctx *ctx, const double *moments, double mu, double *rho,
                      double *energies, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as sq_density_energy, with the same arguments and synchronisation,
 * computed without the context's quadrature-weight and reduction buffers.
 * The per-node weights are formed in registers from moments and the
 * coefficient table, and the reduction partials and sums live in a fixed
 * library-owned device array (a static __device__ array of 3 * 1024 + 4
 * doubles, about 24 KiB, one per GPU, held until the process ends; its size
 * does not depend on the cell).  The call allocates nothing.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other host
 * threads or streams) race and must be serialised by the caller.  rho may
 * differ from sq_density_energy's only by rounding. */
int sq_density_energy_static(sq_ctx *ctx, const double *moments, double mu, double *rho,
                             double *energies, void *stream);

/* Nonlocal atomic forces (Sec. 3.4, nonlocal component, with the FD gradient
 * of Sec. 3.1): forces (host, natom x 3 FP64, Ha/Bohr, row per atom in the
 * order of sq_setup's atom_xyz) =
 *   f_I = -4 sum_{I' images of I} sum_q gamma h^3 p_{I'}(q) p_{I'}^T grad_{h,q} u_q,
 *   u_q = sum_{j=0}^{n_pl} c_q^j t_q^j,
 * with the recurrence run to n_pl (twice the density's length) at the
 * current bounds and the Chebyshev coefficients c_q^j of the Fermi function
 * at Fermi level mu (from sq_fermi_level).  FP64 in both precision modes.
 * Requires bounds (SQ_ESTATE otherwise) and n_pl <= 256 (SQ_EINVAL
 * otherwise).  Uses the workspace's vector buffers; synchronises `stream`. */
int sq_nl_forces(sq_ctx *ctx, double mu, double *forces, void *stream);

/* Release the host tables (never touches caller-owned device memory). */
void sq_destroy(sq_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Batched snapshots: one SCF pass (bounds, moments, Fermi level, density and
 * energies at fixed V_eff, Sec. 3.2-3.3) of many independent snapshots per
 * call, e.g. the configurations of a molecular-dynamics ensemble.  The nodes
 * of all snapshots are cut into blocks; a persistent launch per cube size
 * takes (snapshot, block) items from a device work queue, largest work first.
 * The Fermi level of every snapshot is found on the device by the same Brent
 * iteration as sq_fermi_level (bit-identical results), so a whole pass runs
 * without host round trips and can be captured as one hipGraph.
 * ------------------------------------------------------------------------- */
typedef struct sq_batch sq_batch;

typedef struct sq_batch_options {
    int block_nodes;     /* nodes per work item (0: default 32, or the autotuned value) */
    int wg_per_cu;       /* persistent workgroups per compute unit (0: occupancy limit) */
    int use_graph;       /* 1 (default): capture the pass as a hipGraph on the first
                            sq_batch_step and replay it afterwards; 0: plain launches */
    int bounds_every;    /* recompute the Lanczos bounds at least every this many
                            passes (default 1: every pass).  In between, the previous
                            chi and zeta are reused while V_eff has moved by at most
                            half of the margin slack min_q zeta_q margin/(1+margin)
                            since they were computed (V_eff enters H_q as a diagonal:
                            no eigenvalue moves further than max|delta V|); otherwise,
                            or if a moment leaves [-1, 1], the pass computes fresh
                            bounds. */
    int reuse_check;     /* 1 (default): the V_eff change test above runs before
                            bounds are reused; 0: reused bounds are trusted (for
                            callers that bound the change of V_eff themselves), and a
                            pass in which a moment leaves [-1, 1] is redone with fresh
                            bounds.  That test only catches escapes the moments
                            amplify past 1, which at low n_pl a moderate escape
                            need not do. */
    int shape;           /* SQ_SHAPE_* bits for the recurrence launches of every cube
                            side that has them (other sides ignore them); 0 (default):
                            one cube column per thread and one plane per barrier.
                            sq_batch_autotune chooses them per launch group. */
} sq_batch_options;

/* Kernel shapes of the batched recurrence launches (bits of sq_batch_options.shape). */
#define SQ_SHAPE_TWO_ROWS 1   /* two y-adjacent cube columns per thread: 21-27-point cubes */
#define SQ_SHAPE_TWO_PLANES 2 /* two cube planes per workgroup barrier in the FP64 Lanczos
                                 and moments sweeps: 21-31-point cubes */

void sq_batch_default_options(sq_batch_options *opt);

/* Group n >= 1 contexts into a batch.  Every context must be bound (sq_bind)
 * and all must share one precision; they are borrowed and must outlive the
 * batch.  moments[i] (device, N_d x (n_pl + 1) FP64) and rho[i] (device, N_d
 * FP64) receive snapshot i's results; n_electrons[i] (host) is its N_e.
 * Pointers are copied.  SQ_ECAPACITY if a context needs four projector chains
 * on a cube wider than 31 points. */
int sq_batch_create(sq_batch **batch, sq_ctx *const *ctxs, int n, double *const *moments,
                    double *const *rho, const double *n_electrons, const sq_batch_options *opt);

/* Device workspace the batch needs (work queues, per-workgroup vector
 * buffers sized for the largest cube, Fermi-level state). */
int sq_batch_query(const sq_batch *batch, size_t *workspace_bytes);

/* Bind a caller-allocated device workspace (256-byte aligned) and upload the
 * work queues.  Synchronises `stream`. */
int sq_batch_bind(sq_batch *batch, void *workspace, size_t bytes, void *stream);

/* One pass of every snapshot at its current V_eff.  mu (host, n) and energies
 * (host, n x 4, as in sq_density_energy) receive the results.  The pass runs
 * on a private stream ordered after `stream`; `stream` waits for it.
 * Synchronises.  Per-snapshot failures are reported as for the single-snapshot
 * calls (the first failing snapshot's status and message). */
int sq_batch_step(sq_batch *batch, double *mu, double *energies, void *stream);

/* Time the candidate tile shapes (block_nodes x wg_per_cu) on a sample of
 * every snapshot's nodes (the first eighth; Lanczos and moments launches
 * together) and keep the fastest; then, at that tile, time every kernel shape
 * (SQ_SHAPE_* combinations) each launch group's cube side has, that group
 * alone, and keep its fastest.  With cache_path (host, may be NULL) the
 * choice is read from / appended to that JSON file, keyed by the device and
 * the batch's cube sizes, chain counts and precision.  Invalidates a captured
 * graph.  Synchronises `stream`. */
int sq_batch_autotune(sq_batch *batch, const char *cache_path, void *stream);

/* Chosen tile shape and the number of work items of the current queues. */
int sq_batch_tiles(const sq_batch *batch, int *block_nodes, int *wg_per_cu, int *n_items);

/* Launch group i of the batch (one per cube side and chain count, 0 <= i <
 * *n_groups): its cube side, projector chains and SQ_SHAPE_* bits.  Any
 * output may be NULL.  i < 0 writes only n_groups; SQ_EINVAL if i >=
 * n_groups. */
int sq_batch_group(const sq_batch *batch, int i, int *cube, int *nch, int *shape, int *n_groups);

/* Release host state and the private stream and graph. */
void sq_batch_destroy(sq_batch *batch);

/* Message for the last failure on the calling thread ("" if none). */
const char *sq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SQ_H */
