/*
 * helm.h -- C ABI of an MI355X (gfx950) solver for the heterogeneous Helmholtz equation
 * -Laplace u - k^2 u = f,  k = omega / c  (paper Sec. 1, eq. helm1), in 2-D (5-point
 * stencil) or 3-D (7-point stencil), truncated by a PML (Sec. 2.1-2.2), solved by
 * right-preconditioned GMRES (Sec. 2.3) with Stolk's double-sweep domain-decomposition
 * preconditioner P: J strips along x, each padded with PML at its internal sides and
 * coupled by single-layer-potential transmission sources (eqs. solve_upward and
 * solve_downward), forward sweep j = 1..J, residual, backward sweep J..1.
 *
 * Grids and layouts
 *   interior grid  n_x x n_y (x n_z) points, spacing h;  padded grid  N_x x N_y (x N_z),
 *   N = n + 2*pml_outer.  In 3-D the subdomains are slabs along x (padded planes at
 *   their internal faces) and every field row below is a (z, y) pair, row = z * N_y + y.  The unknowns of the discrete system are all padded-grid points;
 *   an outer PML of pml_outer cells surrounds the interior on all four faces, with
 *   homogeneous Dirichlet values beyond it.
 *   Fields (rhs, u, P-apply input and output) are complex128, interleaved re/im doubles
 *   (the layout of torch.complex128), indexed [rhs][y][x] ([rhs][z][y][x] in 3-D) on the
 *   PADDED grid, x fastest.  The medium c is real float64 on the INTERIOR grid, [y][x]
 *   ([z][y][x]), x fastest; the padded medium takes the value of the nearest interior
 *   point.
 *
 * Memory ownership
 *   The caller owns every array it passes.  Arrays documented "device" live on the
 *   handle's HIP device (normally torch tensors); arrays documented "host" are ordinary
 *   host memory.  The handle owns the strip factors and all workspaces and frees them in
 *   helm_destroy.  All device work is queued on opts.stream (a hipStream_t; NULL = the
 *   default stream).  Calls that return scalars to the host (iteration counts, residuals)
 *   synchronise that stream.
 *
 * Errors
 *   Every entry point returns a helm_status; nothing is thrown across the ABI.  A
 *   human-readable message for the last failure on a handle is in helm_last_error.
 *   HELM_EINVAL leaves the handle usable; HELM_EHIP means a HIP runtime call failed.
 *
 * Threading: a handle may be used by one host thread at a time.
 */
#ifndef HELM_H
#define HELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helm_problem* helm_t;

typedef enum {
    HELM_OK = 0,
    HELM_EINVAL = 1,     /* invalid argument or geometry                          */
    HELM_ENOMEM = 2,     /* device allocation failed                              */
    HELM_EHIP = 3,       /* HIP runtime error                                     */
    HELM_ESTATE = 4,     /* call order: solve / apply before helm_factor          */
    HELM_ESINGULAR = 5,  /* zero or non-finite pivot while factoring a strip      */
    HELM_ENOCONV = 6     /* GMRES did not reach the tolerance within max_iter     */
} helm_status;

typedef enum { HELM_C128 = 0, HELM_MIXED_C64 = 1 } helm_precision;
typedef enum { HELM_FULL = 0, HELM_REDUCED = 1 } helm_mode;

typedef struct {
    int dim;            /* 2, or 3 (7-point stencil, slabs along x)                       */
    int n[3];           /* interior points n_x, n_y, n_z (n_z used when dim = 3)          */
    int pml_outer;      /* outer PML width in cells, all faces (>= 1)                     */
    int pml_iface;      /* interface PML width w: pads on internal strip sides (>= 1)     */
    double pml_power;   /* profile sigma(xi) = sigma_max (xi / (w h))^power; default 2    */
    double pml_s0;      /* outer PML: sigma_max = pml_s0 * c_ref / (w_out h); default 10.
                           The outer PML is part of the global operator A, so it changes
                           the solution u                                               */
    double pml_cref;    /* c_ref; <= 0 selects max(c)                                     */
    const int* beta;    /* host; NULL, or J-1 interface columns (0-based padded-grid
                           column where strip j+1 starts, strictly increasing)           */
    int beta_rule;      /* when beta == NULL: 0 = even split of the interior,
                           1 = the paper's rule (eq. define_beta_j)                      */
    int prec;           /* helm_precision: HELM_C128, or HELM_MIXED_C64 = strip factors and
                           sweeps in complex64 (FP32), GMRES/residuals/outer field FP64  */
    int mode;           /* helm_mode: HELM_FULL (GMRES on the whole grid) or HELM_REDUCED
                           (Sec. 2.3 / Algorithms 2-5: GMRES on the interface columns)    */
    int max_iter;       /* GMRES iteration cap; <= 0 selects 200                          */
    int chunk;          /* rows per chunk of the y-partitioned strip solver; 0 = auto
                           (2-D only: a 3-D slab is one chunk)                           */
    void* stream;       /* hipStream_t for all device work; NULL = default stream        */
    int graph;          /* 1 (default): in REDUCED mode, capture one application of
                           Algorithm 3 per right-hand-side count into a HIP graph and replay
                           it in every GMRES iteration (its input is first copied into a
                           fixed buffer); 0: launch kernel by kernel.  Graphs are not used
                           while kernel timing is enabled                               */
    double pml_iface_s0; /* interface pads: sigma_max = pml_iface_s0 * c_ref / (w h);
                           < 0 (the default) selects 2.5 w, i.e. the same damping per cell
                           sigma_max h / c_ref = 2.5 for every pad width.  The pads belong
                           only to the strip operators A^(j) (Sec. 2.1, definition of
                           Omega^(j)), i.e. to the preconditioner P: they change the
                           iteration count, never the solution                          */
    int sweep;          /* 0 (default): the double sweep P of the paper, upward then
                           downward on the residual (Sec. 2.1).  1: the concurrent double
                           sweep P_c (the paper's remark that both sequences can run at the
                           same time, Sec. 1 and 3.1, in a 2-D form with no crossing point):
                           an upward sweep on f, a downward sweep on f on a stream of its
                           own, and the strip solves of f on D^(j) and D~^(j) (sources both
                           sweeps contain) on a third; P_c f = v + w' - z on every core.
                           Half the sequential depth and 1.5 times the strip solves of P,
                           exact for media that do not vary with x, weaker than P where they
                           do.  Its reduced form keeps the columns beta_j - 1, beta_j        */
    int transmission;   /* 0 (default): PML transmission, the strips padded with PML
                           (Sec. 2.1).  1: Robin transmission, the comparison method of
                           Sec. 4.4: subdomains D^(j) plus the extra column, unpadded, with
                           first-order absorbing conditions d_n u + i k u on their internal
                           sides; a ghost column beyond each side is eliminated, which adds
                           -alpha_x(b) alpha_x(b +- 1/2) rho / h^2, rho = (1 + i k h/2) /
                           (1 - i k h/2) with k at the side's column b, to that column's
                           diagonal and puts the neighbour's data (V_o - rho V_i) / h^2 on
                           it.  With sweep 1 the concurrent sweeps of Sec. 3.1 instead: step
                           n = 1..J solves D^(n) and D^(J+1-n) from f on their cores and
                           the Robin data of both neighbours' latest solutions (none for a
                           neighbour not yet solved), both right-hand sides formed before
                           either solve, so where the chains meet each takes the other's
                           data from the step before; P f takes every core from its
                           subdomain's last solution.  2-D and HELM_FULL only (else
                           HELM_EINVAL); pml_iface and pml_iface_s0 are then unused          */
    int restart;        /* GMRES cycle length (basis vectors kept before a restart); 0
                           (default): 60 in HELM_REDUCED, 30 in HELM_FULL, whose basis
                           vectors are whole fields.  Capped at max_iter                     */
    int batch_fuse;     /* 1: in helm_solve_batch, fuse this problem's strip solves with
                           those of the other problems that set it (multi-problem launches,
                           lockstep rounds; see helm_solve_batch).  0 (default): its own
                           thread and stream                                                  */
} helm_opts;

/* Default options for a 2-D problem of n_x x n_y interior points. */
void helm_default_opts(helm_opts* o, int n_x, int n_y);

/*
 * Algorithm 1, first half (Sec. 2.3): validate the geometry, partition the x axis into J
 * strips (interfaces at half-points, Sec. 2.2), build the PML tables (Sec. 2.1, 2.2) and
 * upload the medium.
 *   c      host, n_y*n_x float64 wave speed (> 0, finite), [y][x]
 *   omega  angular frequency (> 0);  h  grid spacing (> 0);  J >= 1 strips
 *   out    receives the new handle (NULL on failure)
 *   c      (3-D: n_z*n_y*n_x, [z][y][x])
 * HELM_EINVAL: J < 1, a strip core narrower than 2 columns, an interface column with a
 * neighbour inside the outer PML, a padded strip wider than 64 columns, a 3-D slab block
 * (padded width x N_z) above 8192, c <= 0 or not finite, omega or h <= 0, dim not 2 or 3.
 */
helm_status helm_setup(const double* c, double omega, double h, const helm_opts* opts,
                       int J, helm_t* out);

/*
 * Algorithm 1, second half: factor every padded strip operator A^(j) (Sec. 2.2, grid of
 * eq. grid_A_j).  Each strip is block-tridiagonal along y with W x W blocks; it is cut
 * into chunks of opts.chunk rows whose last row is a separator; every chunk is factored
 * by block LU with explicit inverses and its two spikes, and the separators by block LU
 * of their Schur complement.  In 3-D a slab is block tridiagonal along y with dense
 * (W N_z) x (W N_z) blocks (the (x, z) planes); each is inverted by blocked Gauss-Jordan
 * elimination, plane after plane (the blocks of all slabs of one plane together).  2-D:
 * computed in FP64, stored in FP64 (HELM_C128) or rounded to complex64.  3-D HELM_C128:
 * FP64 with partial pivoting over the whole column.  3-D HELM_MIXED_C64: complex64 with
 * FP32 accumulation over column blocks of 128, each diagonal block inverted in FP64 from
 * its 64 x 64 sub-blocks with pivoting inside those only; if a diagonal block is singular
 * or its 1-norm condition exceeds 1e6 the factorisation is redone by the FP64 route and
 * rounded (helm_get_factor_path tells which ran; the environment variable
 * HELM_FACTOR3_FP64=1 selects that route from the start).  Strips or slabs with identical
 * operators share one factorisation in every mode (helm_get_factor_slots).
 * HELM_ESINGULAR if a pivot is zero or not finite, or (2-D) if a block inverted in the
 * factorisation has a 1-norm condition estimate ||S||_1 ||S^-1||_1 above 1e13 (numerically
 * singular in FP64: the strip operator is at or near a resonance, e.g. without PML).
 */
helm_status helm_factor(helm_t H);

/*
 * Autotuner of the strip solver's y-partition (2-D): for each candidate number of rows
 * per chunk, refactor and time `reps` applications of the operator one GMRES iteration
 * applies (Algorithm 3 on the reduced columns of `rhs` in REDUCED mode, A P on `rhs` in
 * FULL mode) with HIP events on the handle's stream; the handle is left factored with
 * the fastest candidate.  The chunk size changes only the order of the substitutions
 * (the strip inverse is the same in exact arithmetic), so any candidate is correct.
 *   rhs     device, nrhs * N_y * N_x complex128 (padded grid): the panel to time on
 *   cand    host, ncand ints >= 2: candidate rows per chunk
 *   best    host, one int (may be NULL): the chosen rows per chunk
 *   ms      host, ncand doubles (may be NULL): milliseconds per application
 * 3-D handles have one chunk per slab: nothing is timed, best = N_y, ms = 0 (factored if
 * it was not).  HELM_EINVAL for nrhs, ncand or reps < 1, a candidate below 2 or a null
 * rhs / cand; errors of helm_factor are passed on.
 */
helm_status helm_autotune(helm_t H, int nrhs, const void* rhs, const int* cand, int ncand,
                          int reps, int* best, double* ms);

/*
 * Algorithm 5: solve A u = f for nrhs right-hand sides by right-preconditioned GMRES
 * with the double-sweep preconditioner, starting from u = 0 (FULL) or u = u~ (REDUCED,
 * Algorithm 2), stopping when the GMRES residual has dropped by `tol` relative to its
 * start (Sec. 4: reduction by 1e-6, capped at tol ||f||), then checking the true
 * residual ||f - A u|| / ||f|| in FP64 and, while it exceeds tol, running another GMRES
 * cycle on that residual r (iterative refinement; right-hand sides that already meet tol
 * take no part), up to max_iter applications of the preconditioner in total.  In REDUCED
 * mode such a cycle starts from u~ = P r instead of the strip solves of Algorithm 2:
 * r - A P r lives on the same interface columns (Sec. 2.1), and the sweep also removes
 * what the complex64 strip solves leave off those columns.  HELM_MIXED_C64 ends its first
 * cycle at three times the rounding noise that Algorithm 2 leaves off the reduced columns
 * (the true residual cannot fall below about that level before the restart), measured
 * per right-hand side in each solve, so that a solve does not depend on earlier ones.
 * When the first cycle ran 16 or more iterations, a later cycle also keeps
 * its new directions orthogonal to the images of the previous cycle's Krylov basis and
 * minimises over both spaces (Krylov recycling; fewer iterations, same stopping rule).
 *   rhs     device, nrhs * N_y * N_x complex128 (padded grid)
 *   u       device, same shape, output
 *   iters   host, nrhs ints (may be NULL): GMRES iterations of every cycle, the paper's
 *           count (Sec. 4); the applications of P that start a REDUCED restart, like
 *           Algorithm 2 and 4, are not iterations (helm_get_stats counts every application)
 *   relres  host, nrhs doubles (may be NULL): explicit ||f - A u|| / ||f||
 * HELM_ESTATE before helm_factor; HELM_ENOCONV if some right-hand side missed tol after
 * max_iter (u and relres still hold the best iterate).
 */
helm_status helm_solve(helm_t H, int nrhs, const void* rhs, void* u, double tol,
                       int* iters, double* relres);

/*
 * Several independent problems solved concurrently (uneven grids, e.g. a batch of
 * different sizes): problem p solves nrhs[p] right-hand sides rhs[p] into u[p] as
 * helm_solve(H[p], ...) would, each driven by its own host thread on its handle's stream,
 * so that the kernels of different problems share the GPU (give each handle its own
 * stream: handles that share a stream are serialised).  Problems whose options set
 * batch_fuse (2-D, HELM_MIXED_C64, the double sweep; at least two of them, on one device,
 * kernel timing off) fuse their strip solves instead: their threads meet in lockstep
 * rounds, one strip solve of each per round, and a round launches the strips of up to 8
 * problems as one launch per strip-solver phase (panels of more than 4 right-hand sides on
 * the two-level separator solve, grouped by the form of phase C; other strip solves of the
 * round launch one by one) on a stream of the call's own, ordered against each problem's
 * stream by events; their reduced operator runs kernel by kernel, not from its graph.
 * Every kernel treats each problem alone, so the results are bitwise those of helm_solve.
 * The call returns when every problem has finished.
 *   H, nrhs, rhs, u   host arrays of nprob entries; rhs[p], u[p] device fields of H[p]
 *   iters, relres     host, sum(nrhs) entries each (may be NULL), problem by problem
 * Returns HELM_OK when every problem succeeded, else the status of the first failing
 * problem (its message in helm_last_error(H[p])).  The handles must be distinct.
 */
helm_status helm_solve_batch(int nprob, const helm_t* H, const int* nrhs, const void* const* rhs,
                             void* const* u, double tol, int* iters, double* relres);

/*
 * Misfit and its gradient with respect to the squared slowness m = 1/c^2 on the interior
 * grid (the adjoint-state method; the paper has no gradient, this is the differentiation
 * form of its solver).  For sources f_s, receivers R and data d_s:
 *   J = 1/2 sum_s ||R u_s - d_s||^2,      A u_s = f_s,
 *   dJ/dm_p = omega^2 Re sum_s sum_{q -> p} conj(lambda_s[q]) u_s[q],
 *   A^H lambda_s = R^T (R u_s - d_s),
 * where q runs over the padded points whose medium is that of interior point p (p itself,
 * plus the outer-PML points behind an edge point).  Only the -k^2 u term of A depends on m.
 * The adjoint systems use the same factors: the PML operator is A = D S with
 * D = alpha_x(x) alpha_y(y) and S complex symmetric (Sec. 2.2), so
 * conj(lambda) = A^{-1}(D conj(q)) / D.  The PML itself (its reference speed fixed at
 * helm_setup) is held constant.  Both solves follow helm_solve with tolerance tol.
 *   src     device, nsrc * N_y * N_x complex128, [source][y][x] (padded grid)
 *   rec     device, nrec int64: flat padded-grid indices y * N_x + x of the receivers
 *           (a receiver listed twice counts twice)
 *   d       device, nsrc * nrec complex128, [source][receiver]
 *   misfit  host, one double (output)
 *   grad    device, n_y * n_x doubles, [y][x] interior grid (output, overwritten)
 *   iters   host, 2 * nsrc ints (may be NULL): forward then adjoint GMRES iterations
 * The call allocates and frees its own work arrays (3 * nsrc fields).  2-D problems only.
 * HELM_EINVAL for a 3-D handle, a receiver index outside [0, N_x N_y) or nsrc, nrec < 1; HELM_ESTATE before helm_factor;
 * HELM_ENOCONV if a solve misses tol (misfit and grad are still written).
 */
helm_status helm_grad(helm_t H, int nsrc, const void* src, int nrec, const int64_t* rec,
                      const void* d, double tol, double* misfit, double* grad, int* iters);

/*
 * The preconditioner alone (Sec. 2.1, end): out = P f = v + w for nrhs fields, computed
 * in the handle's precision (opts.sweep = 1: P_c f = v + w' - z).  f, out: device,
 * nrhs * N_y * N_x complex128.
 */
helm_status helm_apply_P(helm_t H, int nrhs, const void* f, void* out);

/*
 * Algorithm 3 on the reduced unknowns (Sec. 2.3): out = (A P psi) restricted to the
 * columns beta_j, beta_j + 1 of every internal interface.  psi, out: device,
 * nrhs * N_y * 2(J-1) complex128, [rhs][y][interface column], interface columns ordered
 * beta_1, beta_1+1, beta_2, beta_2+1, ...  With opts.sweep = 1: (A P_c psi) on the
 * columns beta_j - 1, beta_j, ordered beta_1 - 1, beta_1, beta_2 - 1, ...
 */
helm_status helm_apply_AP_reduced(helm_t H, int nrhs, const void* psi, void* out);

/*
 * A GMRES restart's reduced right-hand side in the reduced form: b = (r - A P r) on the
 * columns beta_j, beta_j + 1 of every internal interface, for a full field r, computed from
 * both sweeps of P in the target-only form of Algorithm 3 (the support statement of Sec. 2.1:
 * r - A v vanishes off beta_j - 1, beta_j and r - A P r off beta_j, beta_j + 1).  r: device,
 * nrhs * N_y * N_x complex128; b: device, nrhs * N_y * 2(J-1) complex128 ordered as in
 * helm_apply_AP_reduced.  HELM_EINVAL for J = 1, the concurrent sweeps or the Robin
 * transmission; HELM_ESTATE before helm_factor.
 */
helm_status helm_restart_rhs_reduced(helm_t H, int nrhs, const void* r, void* b);

/*
 * The FP64 PML stencil (Sec. 2.2): out = f - A u, or out = A u when f is NULL.
 * u, f, out: device, nrhs * N_y * N_x complex128.
 */
helm_status helm_apply_A(helm_t H, int nrhs, const void* u, const void* f, void* out);

/*
 * One padded strip solve x = A^(j)^{-1} r with the stored factors (strip = 0..J-1).
 * r, x: device, nrhs * N_y * W_j complex128, [rhs][y][strip-local column].
 */
helm_status helm_strip_solve(helm_t H, int strip, int nrhs, const void* r, void* x);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): helm_strip_solve without any
 * allocation.  The strip solver's workspace is a static 64 MiB device array of the
 * library, one per GPU, held until the process ends, instead of a buffer of the handle;
 * the factors are those helm_factor stored.  Same arguments, layout and result as
 * helm_strip_solve (the same kernels).  The workspace holds 64 MiB: a 2-D strip solve needs
 * nrhs * N_y * 64 complex values (8 B in HELM_MIXED_C64, 16 B in HELM_C128), a 3-D slab
 * solve (N_y + 2) * Bp * (nrhs rounded up to 16) values (Bp = padded slab block); larger
 * calls return HELM_EINVAL without launching anything.  The handle's device must be
 * current (HELM_EINVAL otherwise).  Every call on one GPU shares that GPU's workspace, and
 * the part a call uses is cleared by a kernel at its start: calls that overlap on one GPU
 * (other streams, other handles, other threads) race and must be ordered by the caller.
 * The call launches kernels only (no allocation, no memset, no event), so it may be
 * captured into a HIP graph.  HELM_ESTATE before helm_factor.
 */
helm_status helm_strip_solve_noalloc(helm_t H, int strip, int nrhs, const void* r, void* x);

/* N_x, N_y, N_z (1 in 2-D) and J. */
helm_status helm_get_dims3(helm_t H, int* N_x, int* N_y, int* N_z, int* J);

/* Geometry queries: N_x, N_y; the J+1 interface columns beta (host, beta[0] = 0,
 * beta[J] = N_x); the first global column and width of each padded strip (host, J each). */
helm_status helm_get_dims(helm_t H, int* N_x, int* N_y, int* J);
helm_status helm_get_partition(helm_t H, int* beta, int* strip_first, int* strip_width);

/* Number of factorisations the handle stores (host int) and, if strip_slot is not NULL,
 * the slot each of the J strips uses (host, J ints, slots numbered by first use).  Strips
 * whose operators
 * coincide (the same width, PML tables and reduced-form target columns, and the same k^2
 * on every row of corresponding columns: e.g. the interior strips of one width in a medium
 * that does not vary with x; the paper notes that a constant medium needs one
 * factorisation, Sec. 4.3) share one; so do 3-D slabs (the same comparison over every
 * z-plane).
 * HELM_ESTATE if helm_setup did not complete. */
helm_status helm_get_factor_slots(helm_t H, int* slots, int* strip_slot);

/* Which factorisation produced the stored 3-D slab inverses (host int):
 *   1  complex64 blocked Gauss-Jordan with pivoting inside the 64 x 64 diagonal
 *      sub-blocks (HELM_MIXED_C64, every diagonal block inverted with a 1-norm
 *      condition <= 1e6),
 *   0  FP64 Gauss-Jordan with partial pivoting over the whole column (HELM_C128, a
 *      complex64 attempt that met a singular or ill-conditioned diagonal block, and 2-D).
 * HELM_ESTATE before helm_factor. */
helm_status helm_get_factor_path(helm_t H, int* path);

/* y-partition of the strip solver: rows per chunk (the last row of every chunk but the
 * last is a separator) and the number of chunks (host ints). */
helm_status helm_get_chunks(helm_t H, int* rows_per_chunk, int* nchunks);

/* Counters of the last helm_solve: applications of the preconditioner (the GMRES
 * iterations of the batch plus one per REDUCED restart; Algorithms 2 and 4 not counted),
 * restarts, and the solve's wall time in milliseconds (host). */
helm_status helm_get_stats(helm_t H, int* ap_applies, int* restarts, double* solve_ms);

/* Panel counters of the last helm_solve (host): right-hand sides that went through the
 * GMRES operator, summed over its applications, and the same sum had converged right-hand
 * sides stayed in the panel.  A right-hand side that has met its target leaves the panel:
 * the unconverged ones are gathered into a panel of the next multiple of 16 (the strip
 * kernels' right-hand-side group), so the strip solves of an application scale with the
 * right-hand sides still iterating; the results are bitwise those of the full panel. */
helm_status helm_get_panel_stats(helm_t H, long long* rhs_applied, long long* rhs_applied_full);

/* Strip-solve counters of the last helm_solve_batch the handle took part in (host):
 * multi-problem launches (one launch per phase for the current strip of up to 8 problems)
 * and strip solves launched on their own.  Both zero when the handle was not fused. */
helm_status helm_get_fusion_stats(helm_t H, long long* fused, long long* unfused);

/*
 * Kernel timing (profiling aid).  While enabled, every launch of the hot kernels is
 * bracketed by a pair of HIP events on the handle's stream (events are recorded
 * asynchronously; no synchronisation is added).  helm_get_kernel_times synchronises the
 * stream and returns, per kernel class, the number of launches and their summed
 * duration in milliseconds since timing was last enabled.  Classes (nclass <= 8):
 *   0 strip solve phase A (chunk substitutions)   1 phase B (separators)
 *   2 phase C (spike correction + scatter)        3 factor, chunks
 *   4 factor, separators                          5 FP64 stencil
 *   6 GMRES vector kernels                        7 other
 * launches, total_ms: host arrays of nclass entries.  At most 65536 launches are
 * recorded per enable; later ones are counted but not timed (ms stays a lower bound).
 * enable is a bit mask of the classes to time (bit c = class c, 0xFF = all); launches of
 * the other classes are still counted.  0 disables timing.  Every timed launch costs two
 * event records on the stream, so timing only the classes of interest disturbs less.
 * While timing is enabled the reduced operator is launched kernel by kernel, not replayed
 * from its graph (the durations of events recorded by graph nodes cannot be read).
 */
helm_status helm_set_kernel_timing(helm_t H, int enable);
helm_status helm_get_kernel_times(helm_t H, int nclass, int* launches, double* total_ms);

const char* helm_last_error(helm_t H);
void helm_destroy(helm_t H);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
