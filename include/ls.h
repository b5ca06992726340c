/*
 * ls.h — C ABI of the MI355X FFT-accelerated Lippmann–Schwinger operator.
 *
 * Method: Anand, Pandey, Rathish Kumar, Paul, "An efficient high-order
 * Nystrom scheme for acoustic scattering by inhomogeneous penetrable media
 * with discontinuous material interface" (arXiv:1509.05063).
 *
 * The library discretises the Lippmann–Schwinger equation (Sec. 1,
 * eq:-Lippmann)
 *
 *     u(x) + kappa^2 int G_kappa(x - y) m(y) u(y) dy = u^i(x),  m = 1 - n^2,
 *
 * on two overlapping patches of a star-shaped scatterer (Sec. 2): a Cartesian
 * interior patch and a boundary band whose transverse parameter t2 = 0 is the
 * material interface.  ls_apply evaluates v = u + kappa^2 K_h u (the operator
 * that GMRES applies every iteration, Sec. 2) in four device steps:
 * projection onto equivalent sources on cell faces (Sec. 3.2,
 * equiv-conv-loc), FFT convolution with the Green's function on the face
 * lattices (Sec. 3.2), interpolation back to the Nystrom nodes through cell
 * Dirichlet fits (Sec. 3.2, eq:-PWE), and a sparse near-field correction
 * that carries the singular and interface quadrature weights (Sec. 3.1,
 * eq:-VolInt-Adj-NonAdj-I).  The subtraction of the adjacent cells'
 * equivalent-source fields from the face values (Sec. 3.2) is linear and
 * touches only pairs the near field stores, so ls_create folds it into the
 * near-field weights once.
 *
 * Conventions shared by every entry point
 *   - Complex vectors are interleaved (re, im).  LS_C128: double, LS_C64:
 *     float.  A block of nrhs vectors is laid out [nrhs][N] (vector-major).
 *   - Device pointers are HIP device memory owned by the caller; host
 *     pointers are ordinary memory owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Points are stored in the operator's own order (sorted by cell); the
 *     caller reads that order with ls_points and works in it.
 *   - Errors are returned as ls_status; no exception crosses the ABI.  The
 *     text of the last error of the calling thread is ls_last_error().
 *     Device faults surface as LS_EDEVICE at the next synchronising call.
 */
#ifndef LS_H
#define LS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LS_OK = 0,
  LS_EINVAL = 1,      /* invalid argument or unsupported parameter combination */
  LS_ENOMEM = 2,      /* host or device allocation failed */
  LS_EDEVICE = 3,     /* HIP runtime error (no device, launch failure, fault) */
  LS_ENOCONV = 4,     /* solver stopped before the tolerance; iterate written */
  LS_EBUDGET = 5,     /* request does not fit the memory budget */
  LS_ENOTREADY = 6,   /* serving ticket not finished yet */
  LS_ENUMERIC = 7     /* non-finite value (NaN / Inf) in the data or during an iteration */
} ls_status;

typedef enum { LS_C128 = 0, LS_C64 = 1 } ls_prec;

/* Scatterer and patches (Sec. 2; the patch layout is a reading, the paper
 * gives none).  Boundary R(theta) = 1 + shape_a cos(shape_k theta).
 *   interior patch: lattice x = h (i1, i2), nodes where its partition of
 *                   unity is positive (s(x) = |x|/R(arg x) < s_b);
 *   boundary patches: x = s R(theta) (cos, sin), s = 1 - (1 - s_in) t2,
 *                   t2 = i2/N2 (0 <= i2 <= N2), interface at t2 = 0;
 *                   n_patches <= 1: one periodic band, theta = 2 pi t1,
 *                   t1 = i1/N1 (0 <= i1 < N1);
 *                   n_patches = P >= 2: P overlapping patches, patch p
 *                   spanning theta in [theta_p - D, theta_p + D] with
 *                   theta_p = 2 pi p / P, D = pi / P + overlap, t1 = i1/N1
 *                   (0 <= i1 <= N1) mapped linearly onto that range;
 *   partition of unity: omega_band = step((s - s_a)/(s_b - s_a)),
 *                   omega_int = 1 - omega_band; with P >= 2 patches a
 *                   boundary node also carries the tangential partition of
 *                   unity b_p / sum_q b_q, b_p = step((D - |theta -
 *                   theta_p|) / (2 overlap)), which vanishes to all orders
 *                   at the patch ends (nodes with zero weight are not
 *                   unknowns). */
typedef struct {
  int dim;            /* 2 (the only value accepted) */
  double shape_a;
  int shape_k;
  double h;
  double s_in;
  int N1, N2;
  double s_a, s_b;
  int n_patches;      /* boundary patches (0 or 1: one periodic band) */
  double overlap;     /* P >= 2: half-overlap of neighbouring patches, radians, in (0, pi / P) */
} ls_geometry;

/* Quadrature and accelerator parameters (names follow the paper).
 *   Q            Newton–Cotes points (transverse, boundary patch); N2 % (Q-1) == 0
 *   P            Lagrange interpolation nodes per axis (even, >= 4)
 *   chi_c0       cut-off chi == 1 on [0, chi_c0]
 *   r_int        interior cut-off radius (physical units)
 *   r1, r2       boundary cut-off radii in grid units of t1 and t2
 *   polar_*      interior polar rule: graded Gauss rho = a s^grade on
 *                [0, chi_c0 r] (n_in nodes), Gauss on the rest (n_out),
 *                trapezoid in theta (n_theta)
 *   band_*       boundary rule in t1: t1 - t1^x = a s^(M+1) (n_in Gauss
 *                nodes) plus Gauss on the cut-off transition (n_out)
 *   cell_h       cell side H = cell_h * h
 *   q            equivalent-source nodes per cell face
 *   n_fb         Dirichlet fit order: Fourier–Bessel modes |n| <= n_fb
 *   coll_factor  collocation points = coll_factor * 4q per source set
 *   skip_tiles   (storage, not the discretisation) nonzero: do not keep the
 *                near-field rows a second time as dense 16-row tiles (in
 *                single and double precision); batched applies then use the
 *                row kernels.  Saves the tiles' memory (about 1.3x the row
 *                weights of each precision) and their set-up time.
 *   fft_refine   0 or 1: the boundary rule's off-grid values come from
 *                P-point Lagrange stencils on the grid.  r in 2..8: the
 *                Fourier refined polynomial interpolation of Sec. 3.1 along
 *                t1 (single periodic band only, N1 <= 4096 with prime
 *                factors 2, 3, 5): every apply refines each t2 line of the
 *                boundary-patch density r-fold by FFT (zero-padded
 *                spectrum) and the t1 stencils read the refined lines.  The
 *                rows then also hold (r - 1) (N2 + 1) N1 refined columns past
 *                the N unknowns, the dense tiles are not built, and the
 *                workspace grows by (r (N2 + 1) N1 + N) elements per
 *                right-hand side.
 *   fft_refine_interior  nonzero (with fft_refine = r >= 2, cell_h = 8):
 *                the interior polar rule's stencils read the r-fold refined
 *                lattice as well: every apply transforms the interior
 *                density on the M x M box of the cells plus two cells per
 *                side (M rounded up to prime factors 2, 3, 5, at most 4096),
 *                forms the r^2 - 1 shifted lattices (phase ramps, inverse
 *                transforms) and runs the interior contraction once per
 *                shift; the rows and the workspace grow by (r^2 - 1) M^2
 *                elements (plus M^2 for the spectra) per right-hand side.
 *   offgrid_shortcut  nonzero (single periodic band): the paper's shortcut
 *                for interior lattice nodes inside the boundary patch (the
 *                remark after eq:-VolInt-Adj-Sing-MultiSplit): the boundary
 *                rule is evaluated at the patch's grid nodes (their values
 *                s kept in the apply's workspace, refined along t1 like the
 *                densities when fft_refine > 1) and interpolated to those
 *                nodes by P x P stencils instead of being evaluated there;
 *                every apply runs those rules first.  Workspace: rf (N2 + 1)
 *                N1 more elements per right-hand side; no dense tiles. */
typedef struct {
  int Q, P;
  double chi_c0, r_int, r1, r2;
  int polar_n_in, polar_grade, polar_n_out, polar_n_theta;
  int band_M, band_n_in, band_n_out;
  int cell_h, q, n_fb, coll_factor;
  int skip_tiles;
  int fft_refine;
  int fft_refine_interior;
  int offgrid_shortcut;
} ls_params;

/* Refractive index callback: writes n^2 at n points (x, y interleaved);
 * on_boundary[i] != 0 marks interface nodes, where the interior limit is
 * expected.  Called on the creating thread during ls_create only. */
typedef void (*ls_n2_fn)(int64_t n, const double* xy, const int32_t* on_boundary,
                         double* n2_out, void* ctx);

typedef struct ls_op ls_op;

/* Device memory provider.  alloc returns device memory of at least `bytes`
 * bytes on the current device, aligned to 256 bytes, or NULL on failure;
 * release gives back a block alloc returned (with its size).  Both are
 * called on the thread that calls into the library, with the op's device
 * current.  A caching allocator (e.g. PyTorch's) can supply the operator's
 * memory this way, so one pool serves both. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, size_t bytes, void* ctx);
  void* ctx;
} ls_allocator;

/* Build the discrete operator for wavenumber kappa on the current HIP device.
 * Set-up (nodes, weights, near-field quadratures, equivalent-source least
 * squares, Green's function spectra) runs on the host with OpenMP; the
 * results are copied to the device once.  The op owns all its memory: every
 * device block it keeps (operator data, the solver scratch of ls_solve
 * without a caller workspace, targets of ls_targets_create) comes from
 * `alloc` when it is not NULL (it is copied; its ctx must stay valid while
 * the op lives), else from hipMalloc; temporary set-up blocks too.
 * Errors: LS_EINVAL (bad geometry/params, kappa <= 0, cell resonance
 * kappa H >= pi sqrt(2), cut-off reach beyond two cells), LS_ENOMEM (also
 * when alloc returns NULL; everything taken so far is released),
 * LS_EDEVICE. */
ls_status ls_create(const ls_geometry* geom, ls_n2_fn n2, void* ctx, double kappa,
                    const ls_params* params, const ls_allocator* alloc, ls_op** out);

/* Release everything the op holds (NULL is accepted). */
void ls_destroy(ls_op* op);

/* Number of unknowns N. */
ls_status ls_num_points(const ls_op* op, int64_t* N);

/* Node coordinates xy[2N] (host) in operator order and, if key != NULL,
 * key[3N] = (patch, i1, i2): patch 0 = interior lattice (i1, i2) = x/h,
 * patch 1 + p = grid indices of boundary patch p. */
ls_status ls_points(const ls_op* op, double* xy, int32_t* key);

/* Device bytes held by the op (operator data, both precisions). */
size_t ls_resident_bytes(const ls_op* op);

/* Sizes of the discretisation (first nout of): N, boundary-patch nodes,
 * occupied cells, cells per axis, near-field CSR rows, CSR entries, padded
 * face-lattice dims Pa, Pb, equivalent-source unknowns per cell U, face
 * values per cell F, interior slots per cell S, near-field window side,
 * column runs of the CSR rows (0 when the run form is not kept), weights
 * stored in the dense 16-row tiles (single precision, zeros included) and
 * of those the ones in columns beyond the rows' adjacent cells. */
ls_status ls_op_stats(const ls_op* op, int64_t* out, int nout);

/* Workspace bytes ls_apply needs for nrhs vectors in precision prec. */
ls_status ls_workspace_size(const ls_op* op, int nrhs, ls_prec prec, size_t* bytes);

/* v = u + kappa^2 K_h u for nrhs vectors ([nrhs][N] complex, device).
 * Asynchronous on `stream`; no host synchronisation.  ws (device, >=
 * ls_workspace_size bytes) is scratch owned by the caller; applies that run
 * concurrently need distinct workspaces.  u and v must not overlap.
 * LS_C64 runs every step in single precision (weights rounded from the
 * double-precision set-up).  The near-field correction runs on a stream of
 * the operator's own, forked from `stream` by an event and joined back
 * into it before the apply's last kernel (so the work enqueued on `stream`
 * is complete exactly when the apply is; stream capture records the fork
 * and the join).  Applies on one op may be issued from several host
 * threads: the fork / join sequence on the op's stream is taken under a
 * lock of the op, so their near fields queue one after another on that
 * stream while their far fields overlap on the callers' streams.
 * Errors: LS_EINVAL, LS_EDEVICE. */
ls_status ls_apply(ls_op* op, const void* u, void* v, int nrhs, ls_prec prec,
                   void* ws, size_t ws_bytes, void* stream);

/* ls_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result as ls_apply, with the workspace taken from a
 * static device array of the library (LS_NOALLOC_SCRATCH_BYTES = 96 MiB per
 * device, held from the first ls_create on that device until the process
 * ends) instead of a caller buffer.  Allocates nothing.  Every call on one
 * device shares that device's array and no call needs it cleared first;
 * calls that overlap in time on one device (any op, any stream) race on it
 * and must be ordered by the caller.  LS_EINVAL when the apply needs more
 * than the array holds (ls_workspace_size tells how much it needs; e.g.
 * about 75 MiB for one single-precision vector at 946k unknowns), or as
 * ls_apply; LS_EDEVICE as ls_apply. */
ls_status ls_apply_noalloc(ls_op* op, const void* u, void* v, int nrhs, ls_prec prec, void* stream);

/* Size of the static scratch of ls_apply_noalloc, in bytes. */
ls_status ls_noalloc_scratch_bytes(size_t* bytes);

/* One ls_apply with its stages in order on `stream` (the near field not
 * forked) and HIP events recorded between them; waits for completion and
 * writes the stage durations (milliseconds) to
 * stage_ms[0..min(nstage,8)-1]: 0 projection (Sec. 3.2, equiv-conv-loc),
 * 1 face-lattice fill, 2 forward FFTs, 3 spectral product, 4 inverse FFTs,
 * 5 adjacency subtraction + cell Dirichlet fit (eq:-PWE) + combine,
 * 6 near field between interior nodes, 7 near field rows of the boundary
 * patch (Sec. 3.1).  Same arguments and errors as ls_apply. */
ls_status ls_apply_profile(ls_op* op, const void* u, void* v, int nrhs, ls_prec prec, void* ws,
                           size_t ws_bytes, void* stream, double* stage_ms, int nstage);

/* Kernel schedules chosen by ls_autotune for one precision. */
typedef struct {
  int fft_col_tile;     /* columns per workgroup of the column transforms */
  int near_variant;     /* interior contraction: 0 double-buffered staging (16 cells per
                           workgroup), 1 single-buffered, 2 / 3 double-buffered with 32 / 64 cells,
                           4 as 3 with each complex product as three real matrix products */
  int csr_variant;      /* boundary-patch rows: 0 four entries per lane, 1 one entry per lane,
                           2 four entries per lane with run-length column storage,
                           3 dense 16-row tiles on the matrix cores (candidate for multiples
                           of 16 right-hand sides), 4 as 3 with three real products per
                           complex product */
  int fft_variant;      /* 0 separate column transforms and spectral product, 1 fused per column tile */
  int fft_row_threads;  /* threads per workgroup of the row transforms (256, 512 or 1024) */
  int fft_col_threads;  /* threads per workgroup of the fused column kernel (256 or 512) */
  double fft_ms;        /* best time of the transform stages with the chosen tile */
  double near_ms;       /* best time of the interior contraction stage */
  double csr_ms;        /* best time of the boundary-patch rows stage */
  double apply_ms;      /* one apply with all choices in place (the near field concurrent
                           with the far field; the last tuning stage times whole applies so
                           and may revise the transform threads, tile and interior variant) */
  int fft_rows_inplace; /* 1: row transforms with one LDS buffer (rows of at most 4096
                           points; half the LDS, two barriers per pass) */
  int near_rows_first;  /* 1: in the concurrent apply the boundary-patch rows run before the
                           interior contraction on the side stream (0: after it) */
} ls_tune_result;

/* Set the kernel schedule for later applies in precision prec (the fields
 * fft_col_tile ... fft_col_threads, fft_rows_inplace and near_rows_first of
 * *sched; the timing fields are ignored), e.g. to force one variant.  The
 * schedule changes which kernels run, not the discrete operator.  Ranges:
 * fft_col_tile 1 ... the LDS limit (LS_EINVAL beyond it), near_variant 0-4
 * (single precision; double precision has one interior kernel and accepts
 * 0), csr_variant 0-4 (single precision; 2 needs the run-length columns, 3
 * and 4 the dense tiles, and fall back to 2 when nrhs is not a multiple of
 * 16; double precision accepts 0 and 3, its dense tiles), fft_variant 0 / 1,
 * fft_rows_inplace 0 / 1 (1 for rows of at most 4096 points),
 * near_rows_first 0 / 1, fft_row_threads 256 / 512 / 1024, fft_col_threads
 * 256 / 512.  LS_EINVAL leaves the schedule unchanged.  Not to be called
 * while applies or solves on op are in flight. */
ls_status ls_set_schedule(ls_op* op, ls_prec prec, const ls_tune_result* sched);

/* The current schedule of precision prec (timing fields zero). */
ls_status ls_get_schedule(const ls_op* op, ls_prec prec, ls_tune_result* sched);

/* Time the candidate schedules of the apply's tunable stages on this
 * operator (each candidate: three applies of a fixed input, best stage time
 * kept) and keep the fastest for later applies in precision prec.  Allocates
 * and frees its own buffers; synchronous.  The choices change which kernels
 * run, not the discrete operator; the near-field row variants sum each row in
 * a different order, so single-precision results may change in rounding.
 * Not to be called while other applies or solves on op are in flight.
 * Errors: LS_EINVAL, LS_ENOMEM, LS_EDEVICE. */
ls_status ls_autotune(ls_op* op, int nrhs, ls_prec prec, void* stream, ls_tune_result* result);

typedef enum { LS_SOLVE_FP64 = 0, LS_SOLVE_FP32_REFINE = 1 } ls_solve_mode;

/* Orthogonalisation of each new Krylov vector: classical Gram–Schmidt applied
 * twice (default) or once. */
typedef enum { LS_ORTHO_CGS2 = 0, LS_ORTHO_CGS1 = 1 } ls_ortho;

typedef struct {
  double tol;           /* stop when ||f - A x|| <= tol ||f|| (per vector) */
  int max_iter;         /* total inner iterations per vector */
  int restart;          /* GMRES(m) restart length */
  ls_solve_mode mode;   /* FP64 GMRES, or FP32 GMRES inside FP64 refinement */
  double inner_tol;     /* relative tolerance of each inner FP32 solve (per vector, an inner
                           solve stops earlier once it has half the reduction still needed
                           to reach tol) */
  int max_outer;        /* refinement steps */
  int use_x0;           /* nonzero: u_tot holds the initial guess */
  ls_ortho ortho;       /* Gram–Schmidt passes (zero-initialised = CGS2) */
  int graph;            /* nonzero: each Arnoldi step (apply, orthogonalisation,
                           normalisation, copy of its Hessenberg column) is
                           captured once as a HIP graph and replayed; graphs
                           are kept with the op per (precision, passes, nrhs,
                           restart, step) and released by ls_destroy.  Results
                           are bitwise those of the eager launches. */
  int profile;          /* nonzero: HIP events around each stage fill
                           ls_solve_stats.stage_us (ignored with graph) */
  int inner_f64_basis;  /* FP32_REFINE only: nonzero keeps the inner solves'
                           Krylov basis and Arnoldi in complex double around
                           the single-precision apply (the apply's input is
                           rounded to single precision, its output widened) */
} ls_solve_opts;

typedef struct {
  int iterations;       /* inner GMRES iterations (max over vectors) */
  int outer;            /* refinement steps taken */
  int converged;        /* vectors that met tol */
  double rel_residual;  /* max over vectors of ||f - A x|| / ||f|| (FP64 apply) */
  double seconds;       /* wall time of the call */
  double apply_seconds; /* host time spent enqueueing operator applies */
  /* device time per stage in microseconds when opts->profile is set (else
   * zero): 0 double-precision applies, 1 single-precision applies (with
   * their precision conversions), 2 Arnoldi orthogonalisation and
   * normalisation, 3 the rest (residuals, refinement updates, the update
   * x += V y) */
  double stage_us[4];
} ls_solve_stats;

/* Device workspace bytes ls_solve needs for nrhs right-hand sides with
 * these options (restart length and mode decide the Krylov basis). */
ls_status ls_solve_workspace_size(const ls_op* op, int nrhs, const ls_solve_opts* opts, size_t* bytes);

/* Solve (I + kappa^2 K_h) u = u_inc for nrhs right-hand sides (device
 * [nrhs][N] complex double) with matrix-free complex GMRES (Sec. 2),
 * Arnoldi on the device.  FP64: basis, apply and Arnoldi in double.
 * FP32_REFINE: inner GMRES solves with a single-precision apply correct the
 * iterate from double-precision residuals; the inner basis is complex float
 * with double-precision block reductions, or complex double with
 * opts->inner_f64_basis.  Synchronous on return.
 * ws: device workspace of at least ls_solve_workspace_size bytes owned by
 * the caller, or NULL: then the op allocates its own scratch on first use
 * and keeps it (through the op's allocator).  Solves on one op run one at a
 * time (a lock of the op; the Givens buffers are the op's).
 * LS_ENOCONV (tolerance not met within max_iter, or a restart cycle that
 * no longer reduces the residual) and LS_ENUMERIC (a non-finite right-hand
 * side, residual or Hessenberg entry; the iteration stops at the last
 * finite step) still write the best iterate and the stats. */
ls_status ls_solve(ls_op* op, const void* u_inc, void* u_tot, int nrhs,
                   const ls_solve_opts* opts, ls_solve_stats* stats, void* ws, size_t ws_bytes,
                   void* stream);

/* ---------------------------------------------------------------------------
 * The field off the scatterer.  Outside the scatterer the Lippmann–Schwinger
 * equation (Sec. 1, eq:-Lippmann) gives the scattered field as
 * u^s = u - u^i = -kappa^2 K[u], with a smooth integrand; the paper plots it
 * around the scatterer (Sec. 4 figures).  It is evaluated with the
 * operator's plain quadrature: the accelerator for the sources in cells not
 * adjacent to the target's cell (the target is fitted like a boundary-patch
 * node of its cell) and a stored row G(|x - y_j|) c_j for the sources in the
 * adjacent cells.  Near the interface (closer than a few grid spacings) the
 * plain rule loses accuracy, as any fixed quadrature of a nearly singular
 * integrand does.
 * --------------------------------------------------------------------------- */
typedef struct ls_targets ls_targets;

/* A set of n target points xy (host, 2n doubles) strictly outside the
 * scatterer and inside the operator's cell box (the axis-aligned box of
 * cells that cover the nodes).  Builds the per-target rows on the host and
 * uploads them.  Errors: LS_EINVAL (a target inside/on the scatterer or
 * outside the box), LS_ENOMEM. */
ls_status ls_targets_create(ls_op* op, int64_t n, const double* xy, ls_targets** out);
void ls_targets_destroy(ls_targets* tg);

/* us [nrhs][n] (device, complex double) = scattered field at the targets
 * for the totals u_tot [nrhs][N] (device, complex double, operator order, as
 * returned by ls_solve).  Asynchronous on `stream`; ws as for an LS_C128
 * apply of nrhs vectors.  Errors: LS_EINVAL, LS_EDEVICE. */
ls_status ls_scattered_field(ls_op* op, const ls_targets* tg, const void* u_tot, int nrhs, void* us, void* ws,
                             size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Serving.  A server owns worker threads (one HIP stream each, on the device
 * current at ls_server_create) and a set of registered scatterers (operator
 * descriptions, keyed by the caller).  A request asks for the total field of
 * one scatterer under the plane wave exp(i kappa (cos a, sin a).x) (Sec. 1,
 * incident field).  Operators are built on first use and stay resident (near
 * weights, projection/interpolation matrices, Green's function spectra) while
 * the HBM budget allows; idle ones are evicted least recently used first.
 * While a scatterer's solve runs, further requests for it queue and become
 * the right-hand sides of its next solve (up to max_batch); solves of
 * different scatterers run concurrently.  A batched solve advances every
 * right-hand side independently and freezes converged ones, so a request's
 * result is bitwise the same alone and in any mix of fewer than 64
 * right-hand sides (larger batches project onto the equivalent sources with
 * other kernels, equal to rounding).  The n2 callback is called
 * from a worker thread when its operator is built.
 * --------------------------------------------------------------------------- */
typedef struct ls_server ls_server;

typedef struct {
  int max_batch;        /* right-hand sides per solve */
  int workers;          /* concurrent solves */
  double tol;           /* as ls_solve_opts */
  int max_iter;
  int restart;
  ls_solve_mode mode;
  double inner_tol;
  int max_outer;
  ls_ortho ortho;
} ls_server_opts;

typedef struct {
  int64_t N;            /* unknowns of the request's operator */
  int batch;            /* right-hand sides in the solve that served it */
  ls_solve_stats stats; /* of that solve */
  double t_submit, t_start, t_done;   /* seconds since ls_server_create */
} ls_request_info;

typedef struct {
  size_t resident_bytes;
  int resident_ops;
  int64_t queued, running, evictions;
} ls_server_info;

/* budget_bytes: device memory for resident operators plus solver scratch
 * (each solve's workspace, ls_solve_workspace_size, and its right-hand
 * sides).  A request whose operator and single-right-hand-side solve alone
 * exceed the budget finishes with LS_EBUDGET.  Errors: LS_EINVAL. */
ls_status ls_server_create(size_t budget_bytes, const ls_server_opts* opts, ls_server** out);
/* Register a scatterer under `key` (arguments as ls_create; the structs are
 * copied, ctx and n2 must stay valid while the server lives).  Errors:
 * LS_EINVAL (duplicate key, bad arguments). */
ls_status ls_server_add_operator(ls_server* s, uint64_t key, const ls_geometry* geom, ls_n2_fn n2, void* ctx,
                                 double kappa, const ls_params* params);
/* Queue a plane-wave request (incidence angle alpha) for scatterer `key`;
 * returns at once with a ticket.  Errors: LS_EINVAL (unknown key). */
ls_status ls_server_submit(ls_server* s, uint64_t key, double alpha, int64_t* ticket);
/* LS_ENOTREADY while the request is queued or running.  When done: the solve's
 * status (LS_OK, LS_ENOCONV with the best iterate, or its error); u_tot (host,
 * >= 2N doubles = cap, may be NULL) receives the total field in the
 * operator's point order, info (may be NULL) the timings and solve stats. */
ls_status ls_server_poll(ls_server* s, int64_t ticket, double* u_tot, int64_t cap, ls_request_info* info);
/* Forget a finished request. */
ls_status ls_server_release(ls_server* s, int64_t ticket);
/* Node coordinates (2N doubles) of a scatterer's operator once it has been
 * built (LS_ENOTREADY before). */
ls_status ls_server_points(ls_server* s, uint64_t key, double* xy, int64_t cap, int64_t* N);
ls_status ls_server_stats(ls_server* s, ls_server_info* info);
/* Stop the workers (after their running solves), release every operator. */
void ls_server_destroy(ls_server* s);

const char* ls_status_str(ls_status s);
const char* ls_last_error(void);

/* ------------------------------------------------------------------------
 * Three-dimensional face-lattice convolution (the FFT step of the 3-D
 * method, Sec. 3.2, equiv-conv-loc).  In 3-D each source set of a cubic cell
 * lattice lives on a lattice of na x nb x nc nodes indexed [a][b][c] =
 * (normal, tangential, tangential) with spacings hn, ht, ht.  For every set
 *   F(x) = sum over nodes y != x of G(x - y) sigma_m(y) + D(x - y) sigma_d(y)
 * with G(r) = exp(i kappa r) / (4 pi r) and D = dG(|x - y|)/dy along the
 * normal axis (the K(0) = 0 convention), computed by zero-padded FFTs
 * (padded sizes next 2^i 3^j 5^k >= 2n - 1; spectra computed once in double
 * and kept in single precision, one octant of each: the monopole spectrum is
 * even per axis, the dipole one odd along the normal axis and even along the
 * other two).  Single precision (LS_C64) only.  Only this step of the 3-D
 * method is built.
 * ------------------------------------------------------------------------ */
typedef struct ls_conv3d ls_conv3d;

/* LS_EINVAL for non-positive sizes, spacings or kappa, nsets > 1024, or
 * lattices whose padded sizes exceed what one workgroup transforms in LDS
 * (Pc <= 2048, Pb <= 512 tangential, Pa <= 128 normal); LS_ENOMEM /
 * LS_EDEVICE on device failures.  Synchronous (uses the null stream once). */
ls_status ls_conv3d_create(int na, int nb, int nc, double hn, double ht, double kappa, int nsets,
                           ls_conv3d** out);

/* padded[3] = (Pa, Pb, Pc); ws_bytes = workspace one apply needs
 * (nsets * 2 * Pa * (Pb * Pc + 512) complex float: room for any plane
 * skew); resident_bytes = device memory the object holds (spectra,
 * twiddles).  Any pointer may be NULL. */
ls_status ls_conv3d_info(const ls_conv3d* c, int* padded, size_t* ws_bytes, size_t* resident_bytes);

/* sigma: device [nsets][2][na][nb][nc] complex float (kind 0 monopole,
 * kind 1 dipole strengths); field: device [nsets][na][nb][nc] complex float
 * (written); ws: device workspace of at least ws_bytes (caller-owned;
 * concurrent applies need separate workspaces).  Asynchronous on `stream`.
 * LS_EINVAL for null pointers or a short workspace. */
ls_status ls_conv3d_apply(ls_conv3d* c, const void* sigma, void* field, void* ws, size_t ws_bytes, void* stream);

/* Time candidate schedules of the apply on ws (cleared first) and keep the
 * fastest: the plane skew of the workspace layout (0, 32, 64, 512 complex
 * values of padding after each normal-axis plane), columns (4 ... 64) and
 * threads (256, 512) per workgroup of the fused normal-axis pass, columns
 * (4, 8, 16) per workgroup of the second-axis passes.  schedule[4] (may be
 * NULL) receives (normal tile, threads, second tile, skew).  Synchronous on
 * `stream`; LS_TUNE_LOG set in the environment prints every candidate's
 * time to stderr.  The default schedule (16, 256, 8, 0) is used until this
 * is called. */
ls_status ls_conv3d_autotune(ls_conv3d* c, void* ws, size_t ws_bytes, void* stream, int* schedule);

/* Set the schedule[4] (same order as ls_conv3d_autotune's): normal-axis
 * tile 1 ... 64, threads 256 or 512, second-axis tile 1 ... 16 (tiles
 * within 160 KB of LDS), skew 0 ... 512; LS_EINVAL otherwise (the schedule
 * is then unchanged). */
ls_status ls_conv3d_set_schedule(ls_conv3d* c, const int* schedule);

void ls_conv3d_destroy(ls_conv3d* c);

/* ------------------------------------------------------------------------
 * Dense three-dimensional complex FFT (the zero-padded equivalent-source
 * grid of the 3-D method, Sec. 4, transformed as one cube, e.g. 256^3).
 * In place on a device array [n0][n1][n2] of complex float (n2 fastest),
 * unnormalised: direction +1 computes sum_x a(x) exp(-2 pi i k.x / n),
 * direction -1 the same with exp(+2 pi i k.x / n) (so -1 after +1 returns
 * n0 n1 n2 times the input).
 * ------------------------------------------------------------------------ */
typedef struct ls_fft3d ls_fft3d;

/* LS_EINVAL unless every size is >= 1 with no prime factor other than 2, 3
 * and 5, n2 <= 2048, n1 <= 1204, n0 <= 620 (one workgroup transforms a line
 * or a column tile in LDS) and n0 n1 n2 <= 2^31; LS_ENOMEM / LS_EDEVICE on
 * device failures.  Synchronous (twiddle upload). */
ls_status ls_fft3d_create(int n0, int n1, int n2, ls_fft3d** out);

/* Transform `data` (device, owned by the caller) in place, asynchronously on
 * `stream`.  LS_EINVAL for a null pointer or a direction other than +1 / -1. */
ls_status ls_fft3d_exec(ls_fft3d* f, void* data, int direction, void* stream);

void ls_fft3d_destroy(ls_fft3d* f);

#ifdef __cplusplus
}
#endif
#endif /* LS_H */
