/*
 * exx.h -- C ABI of the MI355X pair-Poisson exact-exchange library.
 *
 * The library evaluates, for a set of localized orbitals phi_i on a periodic
 * orthorhombic grid, the exact-exchange energy and orbital potentials of
 * Ko et al., arXiv:1911.10630:
 *
 *   E_xx = - sum_<ij> w_ij h^3 sum_{r in PE_ij} rho_ij(r) v_ij(r),
 *          w_ii = 1, w_ij = 2 (i != j)                       (Eqs. exx, exx_omega)
 *   D^i(r) = sum_j v_ij(r) phi_j(r)   on the ME sphere of each pair
 *                                                            (Eqs. Dxx_mlwf, Dxx_mlwf_omega)
 *
 * where rho_ij = phi_i phi_j, and v_ij solves the Poisson equation
 * del^2 v = -4 pi rho on the PE sphere of radius R_PE around the grid point
 * nearest the pair midpoint (Eq. pe), with Dirichlet values on the shell
 * R_PE < r <= R_ME from an l <= 6 multipole expansion (Eqs. me, mepole),
 * using the 6th-order central-difference Laplacian (Eq. d2_1) and the
 * boundary-charge form of the reduced system (Eq. pe_mat_red), solved by
 * conjugate gradient (Sec. III.C, Step IV).
 *
 * Units: bohr and hartree.  Grids: [n_orb][Nz][Ny][Nx], x fastest, 0-based
 * (the convention of Eq. l2g); with local boxes (params.box_dims) orbitals
 * and D are [n_orb][bz][by][bx] instead, each on its own box.  The caller applies the hybrid mixing
 * fraction a_x (Eq. hyb); E_xx and D are returned unscaled.
 *
 * Timing fields of exx_stats are HIP-event times; in graph mode only the
 * whole solve is timed that way (prep_ms, cg_ms, guess_ms read -1), and the
 * CG kernel's own span is cg_clock_ms (device wall clock, either mode).
 *
 * Call order: exx_setup -> exx_pairs -> exx_solve -> exx_energy_potential
 * (then exx_pairs or exx_solve again for the next step).  Out-of-order calls
 * return EXX_ESTATE.  No call throws or aborts; every failure returns a
 * status and leaves a message for exx_last_error.  A context is not
 * thread-safe: calls on one context must not overlap.
 */
#ifndef EXX_H
#define EXX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct exx_ctx exx_ctx;

typedef enum {
    EXX_OK = 0,
    EXX_EINVAL = -1,   /* bad argument: null pointer, size, radii, dtype       */
    EXX_ENOMEM = -2,   /* device or host allocation failed                     */
    EXX_EDEVICE = -3,  /* HIP runtime error (message names the call)          */
    EXX_ENOCONV = -4,  /* some pair CG did not reach cg_rtol in cg_max_iter;
                          results are still written, flags in exx_pair_info   */
    EXX_ESTATE = -5    /* call out of order                                    */
} exx_status;

enum { EXX_FP64 = 0, EXX_FP32_REFINE = 1 };                 /* CG arithmetic  */
enum { EXX_F64 = 0, EXX_F32 = 1 };                          /* orbital dtype  */
/* Initial CG guess (Sec. III.C Step IV): zero; the previous step's potential
 * of the same (i, j); polynomial extrapolation over up to three earlier
 * steps; or the learned model (exx_model_init / exx_load_model).  Every mode
 * iterates to the same cg_rtol, so the guess changes iterations, not the
 * converged result. */
enum { EXX_GUESS_ZERO = 0, EXX_GUESS_PREVIOUS = 1, EXX_GUESS_EXTRAP = 2, EXX_GUESS_LEARNED = 3 };

/* Preconditioner of the pair CG.  The paper iterates plain CG (Step IV) and
 * points to preconditioners as the way to cut the CG cost (Sec. IV B).
 * EXX_PRECOND_MG: a symmetric multigrid V-cycle (one damped Jacobi step of
 * the 6th-order operator on the PE sphere before and after; 7-point
 * Laplacians on masked coarse boxes of spacing 2^l h with damped Jacobi
 * smoothing; piecewise-constant transfers).  With EXX_FP64 the residual and
 * the iterate are FP64; with EXX_FP32_REFINE the whole iteration runs in
 * FP32 except the iterate, and the true FP64 residual b - A x replaces the
 * recursive one each time the latter has fallen by 1e3 (inner_rtol is not
 * used).  The stopping rule ||b - A x|| <= cg_rtol ||b|| is unchanged, so
 * results agree with the plain iteration to the CG tolerance. */
enum { EXX_PRECOND_NONE = 0, EXX_PRECOND_MG = 1 };

typedef struct {
    int32_t n_grid[3];      /* Nx, Ny, Nz                                       */
    double  cell[3];        /* orthorhombic cell lengths |L_a| (bohr)           */
    double  r_pair;         /* pair iff minimum-image |C_i - C_j| < r_pair      */
    double  r_pe[2];        /* PE radius: [0] self pairs, [1] non-self pairs    */
    double  r_me[2];        /* ME radius: [0] self pairs, [1] non-self pairs    */
    int32_t fd_half_width;  /* n of Eq. d2_1; only 3 is implemented             */
    int32_t l_max;          /* multipole order; only 6 is implemented           */
    double  cg_rtol;        /* stop when ||b - A x||_2 <= cg_rtol ||b||_2       */
    int32_t cg_max_iter;    /* per pair (FP32_REFINE: total inner iterations)   */
    int32_t precision;      /* EXX_FP64 | EXX_FP32_REFINE                       */
    int32_t orbital_dtype;  /* EXX_F64 | EXX_F32 (phi storage; D uses the same) */
    int32_t guess;          /* EXX_GUESS_*: initial CG guess                    */
    double  inner_rtol;     /* FP32_REFINE: relative tolerance of each FP32 solve */
    int32_t block_threads;  /* CG work-group size; 0 = default choice           */
    int32_t cg_cols;        /* CG columns per thread (z-march); 0 = default;
                               -1 = the flat kernel (any sphere size)           */
    int64_t wave_pairs;     /* max pairs per launch wave; 0 = as many as fit    */
    int32_t keep_intermediates; /* 1: keep rho, b per pair for exx_debug_pair   */
    int32_t autotune;       /* 1 (default): exx_setup times every CG kernel
                               variant that fits (a few CG iterations on a
                               synthetic batch) and keeps the fastest; with
                               n_classes >= 2 the first exx_pairs_spread does
                               it instead, on a batch in its class mix;
                               0: choose by occupancy alone                  */
    int32_t graph;          /* 1: exx_solve captures its launches into a HIP
                               graph on a stream of its own and replays it
                               while the pairs, phi and the model buffers are
                               unchanged (zero or learned guess; the
                               history guesses always run eagerly)           */
    int32_t box_dims[3];    /* orbital storage box (bx, by, bz) in grid points;
                               0 = the whole grid.  Orbital k (and D^k) is
                               stored on the periodic box starting at
                               exx_box_origins()[k] and is zero outside it */
    int32_t precond;        /* EXX_PRECOND_NONE (default) | EXX_PRECOND_MG      */
    /* Per-pair subdomains (the spread- and overlap-dependent domains the paper
     * outlines for its next version, Sec. IV A): n_classes = 0 (default) keeps
     * the two classes above (self pairs on r_pe[0] / r_me[0], all others on
     * r_pe[1] / r_me[1]) and exx_pairs.  n_classes in [2, EXX_MAX_CLASSES]
     * uses the classes class_r_pe[k] / class_r_me[k] (r_pe strictly
     * ascending, r_me - r_pe >= n max(h) each) and exx_pairs_spread, which
     * puts each pair on the smallest class that covers Omega_ij (see there);
     * r_pe / r_me are then ignored.  The learned guess runs on every class
     * with one coarse cube, sized for the largest class. */
    int32_t n_classes;
    double  class_r_pe[4], class_r_me[4];
    double  omega_scale;    /* radius of Omega_i = omega_scale * spread_i      */
} exx_params;

#define EXX_MAX_CLASSES 4

typedef struct {
    int64_t n_pairs;
    int64_t n_self;
    int64_t iters_total;     /* sum of CG iterations (FP32 inner + FP64 outer)  */
    int32_t iters_min, iters_max;
    int64_t n_not_converged;
    double  relres_max;      /* max true relative residual over pairs          */
    double  solve_ms;        /* last exx_solve: all its kernels, HIP events     */
    double  prep_ms;         /* last exx_solve: pair-preparation kernel         */
    double  cg_ms;           /* last exx_solve: persistent CG kernel, summed over
                                waves (HIP events around each launch)          */
    double  dxx_ms;          /* last exx_energy_potential: D kernel, HIP events
                                (pairs in waves: D is summed wave by wave inside
                                exx_solve, and this times only the rounding of
                                the FP64 partial sums)                         */
    double  energy_ms;       /* last exx_energy_potential: E reduction          */
    int32_t solve_grid;      /* persistent work-groups launched                 */
    int32_t solve_block;     /* threads per work-group                          */
    int32_t cg_cols;         /* columns per thread (0: flat kernel)             */
    int32_t cg_bands[2];     /* y bands per class                               */
    int64_t outer_total;     /* FP32_REFINE: FP64 residual passes               */
    int64_t n_pe[2], n_me[2];/* subdomain sizes per class                       */
    int64_t cg_bytes;        /* algorithmic CG bytes of the last solve          */
    int64_t solve_bytes;     /* algorithmic bytes of the whole solve kernel     */
    int64_t dxx_bytes;       /* algorithmic bytes of the D kernel               */
    int64_t device_bytes;    /* device memory held by the context              */
    int32_t n_waves;         /* pair waves of the last solve (1 = one launch)   */
    int32_t wave_n;          /* pairs per wave (the last wave may hold fewer)   */
    int32_t guess_pairs;     /* pairs whose CG started from a non-zero guess    */
    double  guess_ms;        /* last solve: guess kernels / model inference     */
    int32_t tuned;           /* CG variants the autotuner timed (0: none)      */
    double  tune_ms;         /* time of those tuning launches                   */
    int32_t graph_builds;    /* graph mode: captures so far                     */
    int32_t graph_launches;  /* graph mode: solves launched as a graph          */
    int32_t n_classes;       /* subdomain classes in use (2 with n_classes = 0)  */
    int64_t class_n_pe[4], class_n_me[4];  /* sizes per class                  */
    int64_t class_pairs[4];  /* pairs per class in the current list            */
    int64_t class_capped;    /* pairs whose Omega_ij the largest class does not
                                cover (exx_pairs_spread; they use that class)  */
    int32_t cg_inflight[2];  /* planes of loads in flight in the CG kernel's
                                FP64 / FP32 passes (1 or 2)                    */
    int32_t cg_cols32;       /* columns per thread of the FP32 passes          */
    double  cg_clock_ms;     /* last solve: the CG launches' spans, first
                                work-group start to last work-group end on the
                                device wall clock, summed over waves (graph
                                mode included); -1 if unavailable            */
} exx_stats_t;

/* Fills *p with the paper's method defaults (n = 3, l_max = 6, FP64, zero
 * guess, cg_rtol 1e-10, cg_max_iter 20000) and autotune = 1.  Grid, cell and radii are zeroed
 * and must be set by the caller. */
void exx_default_params(exx_params *p);

/* Validates the parameters, builds the self and non-self proto-subdomains
 * (Alg. 2) and uploads their tables to `device`.  EXX_EINVAL if any radius is
 * non-positive, R_ME - R_PE < n * max(h) (the stencil would leave PE u shell,
 * Sec. IV.A), or an unimplemented order is requested.  *out owns every
 * device allocation; free with exx_destroy. */
exx_status exx_setup(const exx_params *p, int device, exx_ctx **out);

/* Builds the unique pair list {i <= j : i == j or |C_i - C_j| < r_pair}
 * (minimum image; Step II) ordered by (i, j), the pair origins (grid point
 * nearest the minimum-image midpoint, Step III) and per-orbital pair lists,
 * and sizes the per-pair device buffers.  The pair search runs on the GPU
 * through a periodic cell list and equals the plain double loop bit for bit.
 * centers: host, [n_orb][3] bohr, copied.  *n_pairs receives the pair count.
 * The pairs are split into waves sized from the device memory free at this
 * call (2 GiB kept free): allocate the orbital and D buffers before it.  A
 * wave holds its pairs' right-hand sides and potentials, each at its own
 * class's size (n_pe rounded up to 64, and n_pe + n_shell, FP64); with
 * more than one wave D's FP64 partial sums ([n_orb][box]) are held too.
 * EXX_ENOMEM if not even one pair fits. */
exx_status exx_pairs(exx_ctx *ctx, int32_t n_orb, const double *centers, int64_t *n_pairs);

/* The pair list of exx_pairs with per-pair subdomain classes
 * (params.n_classes >= 2).  spreads: host, [n_orb] bohr, the orbitals'
 * spreads (for MLWFs, the root of the spread functional's second moment).
 * Orbital i gets the domain Omega_i, the ball of radius
 * R_i = omega_scale * spread_i about C_i; pair (i, j) the domain
 * Omega_ij = Omega_i cap Omega_j (Omega_i for the self pair).  The pair's PE
 * sphere about its origin g must hold Omega_ij; it is taken to need the
 * radius |g - c| + rho, (c, rho) the smallest ball that encloses Omega_ij.
 * With d = |C_j - C_i| (minimum image) and x = (d^2 + R_i^2 - R_j^2) / (2d)
 * the signed distance from C_i to the plane of the spheres' intersection:
 *   d >= R_i + R_j:  empty; radius 0 (the smallest class)
 *   d = 0:           c = C_i, rho = min(R_i, R_j)
 *   x <= 0:          Omega_ij holds a great circle of Omega_i: c = C_i, rho = R_i
 *   x >= d:          the same for Omega_j: c = C_j, rho = R_j
 *   otherwise:       c = C_i + (x / d) (C_j - C_i), rho = sqrt(R_i^2 - x^2)
 * The pair goes to the smallest class whose r_pe is at least that radius,
 * or to the largest class (counted in exx_stats class_capped).  spreads is
 * read during the call.  Everything else is as exx_pairs (same errors).
 * EXX_EINVAL also if n_classes < 2 or a spread is negative or not finite
 * (omega_scale was checked by exx_setup). */
exx_status exx_pairs_spread(exx_ctx *ctx, int32_t n_orb, const double *centers, const double *spreads,
                            int64_t *n_pairs);

/* Subdomain class of each pair of the current list (exx_pair_info order):
 * 0 self / 1 other with n_classes = 0, the class exx_pairs_spread chose
 * otherwise.  cls: host, [n_pairs].  EXX_ESTATE before exx_pairs. */
exx_status exx_pair_class(exx_ctx *ctx, int32_t *cls);

/* Owner of each pair of the current list under Alg. 1 (the refinement of
 * the non-unique list L0 to the unique list Lu that balances the pairs over
 * the orbitals, Sec. III C).  L0 row i holds every orbital overlapping i,
 * itself included, in ascending minimum-image distance from i (squared FP64
 * distance; ties by index).  owner: host, [n_pairs], receives i or j for
 * pair (i, j) in exx_pair_info order (the self pair's owner is i).
 * *sweeps (may be NULL) receives the number of sweeps, the last of which
 * removed nothing.  Computed on the host on first request after exx_pairs
 * (sequential by construction: each removal changes the rows later orbitals
 * scan).  EXX_ESTATE before exx_pairs, EXX_EINVAL if owner is NULL. */
exx_status exx_pair_owners(exx_ctx *ctx, int32_t *owner, int32_t *sweeps);

/* Box origins chosen by exx_pairs, host [n_orb][3] grid points: origin =
 * nearest grid point of the centre minus box_dims / 2 (mod N), or 0 along
 * an axis where the box spans the grid.  exx_pairs returns EXX_EINVAL if an
 * ME sphere of a pair leaves the box of one of its orbitals (D would be cut
 * off): boxes of edge 2 (R_pair / 2 + R_ME) / h + 4 always suffice. */
exx_status exx_box_origins(exx_ctx *ctx, int32_t *origins);

/* Enqueues every pair solve on `stream` (a hipStream_t; NULL = default):
 * gather and pair density (Step III, Eq. l2g), multipole moments
 * (Eq. mepole), shell potential (Eq. me) and right-hand side
 * (Eq. pe_mat_red), conjugate gradient on the stencil of Eq. d2_1 (Step IV),
 * pair energy (Step V, Eq. exx_omega).  phi: device,
 * [n_orb][Nz][Ny][Nx] of orbital_dtype, read-only, must stay valid until
 * the stream work completes.  Asynchronous.  When the pairs' potentials
 * do not fit at once, the pairs run in waves and D is summed wave by wave
 * into FP64 partial sums during this call (results do not depend on the
 * split). */
exx_status exx_solve(exx_ctx *ctx, const void *phi, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): exx_solve
 * with nothing allocated during the call.  The CG work vectors live in a
 * fixed 128 MiB device array that the library defines once per GPU (held
 * from module load until the process ends) instead of the context's
 * buffers; the CG runs on as many work-groups as that array holds slots
 * for (fewer than exx_solve when the subdomains are large), so it can be
 * slower; results are the same bit for bit.  Launches are eager (params.graph
 * is ignored) and only guess = EXX_GUESS_ZERO is accepted (EXX_EINVAL
 * otherwise: the other guesses allocate).  EXX_EINVAL with a message if one
 * CG slot of the current pair list needs more than the array holds.  Every
 * call on one GPU shares that GPU's array, whatever the context: calls that
 * overlap on one GPU race (serialize them).  Nothing in the array needs to
 * start at zero; the previous call's contents are overwritten.  Everything
 * else is as exx_solve (same call order, same ownership, asynchronous on
 * `stream`; the per-wave CG timings of exx_stats are recorded only when an
 * earlier exx_solve on the context created their events). */
exx_status exx_solve_static(exx_ctx *ctx, const void *phi, void *stream);

/* Enqueues D accumulation (Step V, Eq. Dxx_mlwf_omega: D^i += v_ij phi_j
 * and D^j += v_ij phi_i over the ME sphere of each pair) and the E reduction
 * (Eq. exx_omega) on `stream`, then synchronizes it.  dxx: device, same shape and dtype as phi, fully
 * overwritten (every point of every orbital).  *e_xx receives E_xx (host).
 * Returns EXX_ENOCONV (with results written) if any pair failed to
 * converge. */
exx_status exx_energy_potential(exx_ctx *ctx, double *e_xx, void *dxx, void *stream);

/* Counters and timings of the last solve (synchronizes nothing; call after
 * exx_energy_potential). */
exx_status exx_stats(exx_ctx *ctx, exx_stats_t *st);

/* Per-pair results of the last solve, copied to host arrays of length
 * n_pairs (any pointer may be NULL): orbital indices, pair origin grid
 * point [n_pairs][3], pair energy e_ij = h^3 sum rho x, CG iterations,
 * convergence flag, true relative residual. */
exx_status exx_pair_info(exx_ctx *ctx, int32_t *pi, int32_t *pj, int32_t *origin, double *e,
                         int32_t *iters, int32_t *converged, double *relres);

/* Copies one pair's arrays to host buffers (any may be NULL), after a
 * solve: v on PE in the proto-subdomain order of Eq. rbar (n_pe), v on the
 * shell (n_me - n_pe), the 49 real multipole moments Q_lm (index l*l+l+m,
 * real orthonormal harmonics), and, if keep_intermediates was set, the
 * pair density and right-hand side on PE.  EXX_ESTATE if the intermediates
 * were not kept.  Synchronizes the device. */
exx_status exx_debug_pair(exx_ctx *ctx, int64_t pair, double *v_pe, double *v_shell, double *q_lm,
                          double *rho, double *rhs);

/* ---- learned initial guess ------------------------------------------------
 *
 * A 3-D convolutional U-Net (4 levels, 16-64 channels, bf16 weights with
 * FP32 accumulation) maps a pair's right-hand side, averaged onto a cube of
 * coarse cells of `coarsen`^3 grid points around the pair origin, to the
 * coarse potential; the potential is interpolated back onto the PE sphere as
 * the CG starting point (EXX_GUESS_LEARNED).  The paper names better initial
 * guesses as the route to fewer CG iterations (Sec. III.C Step IV, Sec. IV.B).
 * The model lives in the context and survives exx_pairs. */

/* Creates a model with random (He-normal, seeded) weights.  coarsen: 2, 4
 * or 8 grid points per coarse cell edge, else EXX_EINVAL. */
exx_status exx_model_init(exx_ctx *ctx, int32_t coarsen, uint64_t seed);

/* Adam training on the pairs of the last solve: input its right-hand sides,
 * target its converged potentials on ME.  The pairs are those still
 * resident: every pair, or the last wave's when the solve ran in waves (the
 * earlier waves' right-hand sides are released).  epochs >= 1,
 * 1 <= batch <= resident pairs, lr > 0.  *loss receives the mean
 * masked squared error of the last epoch (normalized units: potential over
 * RMS(b) h^2, per coarse cell that meets ME).  epochs = 0 only evaluates
 * that error over every pair, without updating (lr ignored).  Synchronizes
 * `stream`.  The weight-gradient sums use atomics, so training is not
 * bitwise reproducible; inference is. */
exx_status exx_model_train(exx_ctx *ctx, int32_t epochs, int32_t batch, double lr, uint64_t seed, double *loss,
                           void *stream);

/* Serializes the model's FP32 weights into buf (host).  buf NULL: *bytes
 * receives the size.  Else *bytes must hold at least that size (EXX_EINVAL
 * otherwise) and receives it. */
exx_status exx_model_save(exx_ctx *ctx, void *buf, size_t *bytes);

/* Replaces the model by a blob from exx_model_save (host, copied).
 * EXX_EINVAL if the blob's header or size does not match. */
exx_status exx_load_model(exx_ctx *ctx, const void *weights, size_t bytes);

/* Coarse cube edge the model runs at for this context (0 without model). */
int32_t exx_model_edge(const exx_ctx *ctx);

/* One 3x3x3 zero-padded convolution of model layer `layer`, for
 * verification: y[v][co] = sum_tap sum_ci x[v + off(tap)][ci] W[tap][co][ci]
 * with off(tap) = (tap % 3, tap / 3 % 3, tap / 9) - 1 in (x, y, z) and zero
 * outside the cube (transposed = 0), or the input-gradient form with
 * W[26 - tap][co][ci] summed over co (transposed = 1, channel counts
 * swapped).  x: device bf16
 * [n][edge^3][Cin] channels-last, voxel index (z * edge + y) * edge + x;
 * y: device FP32 [n][edge^3][Cout].  Asynchronous on `stream`. */
exx_status exx_model_conv(exx_ctx *ctx, int32_t layer, int32_t transposed, const void *x, float *y, int32_t n,
                          int32_t edge, void *stream);

/* Weight gradient of layer `layer`, for verification: dw[tap][co][ci] =
 * sum_v dy[v][co] x[v + off(tap)][ci].  x, dy: device bf16 channels-last;
 * dw: device FP32 [27][Cout][Cin], overwritten.  Asynchronous. */
exx_status exx_model_wgrad(exx_ctx *ctx, int32_t layer, const void *x, const void *dy, float *dw, int32_t n,
                           int32_t edge, void *stream);

/* ---- measurement -----------------------------------------------------------
 *
 * Streaming rates of plain kernels on `device`, the measured ceiling that the
 * pair CG's HBM bandwidth is set against beside the nominal peak.  Not part
 * of the method.  Five arrays of bytes_per_array bytes (rounded down to a
 * whole number of 16 KiB) are allocated, zeroed and freed inside the call.
 * gbs: host [4] receives GB/s (1e9 bytes per second, every byte read or
 * written counted once) of the best launch of each kind:
 *   gbs[0] read   two arrays read, nothing written
 *   gbs[1] copy   one read, one written
 *   gbs[2] triad  two read, one written (the CG passes' mix, about 2:1)
 *   gbs[3] cg     three read, two written
 * the best over 4, 8 and 16 work-groups of 256 threads per CU, 1, 2 or 4
 * 16-byte accesses per array in flight per thread, plain or non-temporal,
 * `reps` timed launches each after one untimed (HIP events, default stream).
 * detail (may be NULL): host buffer of detail_len bytes receiving a one-line
 * description of the winning launch shapes.  Synchronizes the device.
 * EXX_EINVAL if gbs is NULL, bytes_per_array < 1 MiB or reps < 1;
 * EXX_ENOMEM if the arrays do not fit; EXX_EDEVICE on any HIP error. */
exx_status exx_stream_rates(int device, int64_t bytes_per_array, int32_t reps, double *gbs, char *detail,
                            int32_t detail_len);

/* Message of the last failing call on ctx (or of the last failing
 * exx_setup when ctx is NULL).  Never NULL. */
const char *exx_last_error(const exx_ctx *ctx);

/* Releases every allocation; NULL is ignored. */
void exx_destroy(exx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* EXX_H */
