/*
 * bmg.h -- C ABI of the MI355X geometric-multigrid solver for the H(div)-conforming
 * interior-penalty discretisation of the Brinkman / Darcy equations
 * (Kanschat, Lazarov, Mao, arXiv 1602.04858).
 *
 * Problem (Section 2.2, eq. Brinkman): -mu Lap u + kappa u + grad p = f, div u = 0
 * on the unit square, mu >= 0 (mu = 0 is Darcy), kappa > 0 cellwise constant.
 * Discretisation (Section 2.3): RT_k velocity x discontinuous Q_k pressure on a
 * uniform N x N mesh, interior-penalty form a_h (eq. ipbrinkman) with face penalty
 * 2 mu sigma / h, saddle-point form (eq. Brinkman-weak).  On a Dirichlet side the
 * normal velocity is an essential condition and the tangential one is imposed by
 * the Nitsche terms of eq. (BCh); an open side carries the natural condition.
 * Solver (Section 3): GMRES preconditioned by the V-cycle B_J over the uniformly
 * refined hierarchy N_j = n0 * 2^j, with the symmetric multiplicative vertex-patch
 * Schwarz smoother (eq. smoother-Multiplicative), natural-injection prolongation,
 * its transpose as restriction, and a direct solve on the coarsest mesh.
 *
 * Vector layout ("canonical numbering"), with nb = k+1, N cells per side, cell
 * c = cy*N + cx, basis L_b = orthonormal Legendre on [0,1], psi_0 = 1-t,
 * psi_1 = t, psi_a = int_0^t L_{a-1} (a >= 2):
 *   x-face dofs  (i = 0..N, cy, b)      at (cy*(N+1) + i)*nb + b          [u_x = psi_a(xi) L_b(eta), a = 0/1]
 *   y-face dofs  (j = 0..N, cx, b)      at N(N+1)nb + (j*N + cx)*nb + b   [u_y = L_b(xi) psi_a(eta), a = 0/1]
 *   interior     (c, comp, a >= 2, b)   at 2N(N+1)nb + c*2k*nb + (comp*k + a-2)*nb + b
 *   pressure     (c, a, b)              at n_u + c*nb^2 + b*nb + a         [p = L_a(xi) L_b(eta)]
 * with n_u = 2N(N+1)nb + 2k*nb*N^2 and n_p = nb^2 N^2.  A full vector is the
 * velocity block followed by the pressure block (n_u + n_p doubles).
 *
 * Conventions for every call:
 *   - pointers named *_dev are device pointers (hipMalloc'd or torch tensors)
 *     owned by the caller; *_host are host pointers; nothing is retained after
 *     the call returns unless stated;
 *   - all device work is enqueued on the stream given to bmg_setup; calls that
 *     return host results synchronise that stream;
 *   - a handle is used by one host thread at a time;
 *   - every call returns a bmg_status; on an argument error nothing is modified;
 *     bmg_last_error() gives a message for the last failing call on a handle.
 */
#ifndef BMG_H
#define BMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmg_ctx* bmg_handle;
typedef struct bmg_batch* bmg_batch_handle;

typedef enum {
  BMG_OK = 0,
  BMG_E_ARG = 1,           /* invalid argument (null pointer, out-of-range parameter) */
  BMG_E_UNSUPPORTED = 2,   /* valid but not implemented (e.g. k outside {0,1,2}) */
  BMG_E_NOMEM = 3,         /* workspace too small or device allocation failed */
  BMG_E_HIP = 4,           /* a HIP runtime call failed */
  BMG_E_SINGULAR = 5,      /* a local or coarse matrix could not be inverted */
  BMG_E_NOT_CONVERGED = 6, /* maxit reached; the best iterate is returned */
  BMG_E_NONFINITE = 7,     /* NaN/Inf in inputs or in the iteration */
  BMG_E_STATE = 8          /* call not valid for this handle */
} bmg_status;

enum { BMG_BC_DIRICHLET = 0, BMG_BC_OPEN = 1 };                 /* sides: 0 x=0, 1 x=1, 2 y=0, 3 y=1 */
enum { BMG_P_FP64 = 0, BMG_P_FP32 = 1, BMG_P_BF16 = 2 };        /* preconditioner arithmetic: FP64; FP32;
                                                                   FP32 with bfloat16-stored patch inverses */
enum { BMG_CYCLE_STANDARD = 0, BMG_CYCLE_VARIABLE = 1 };        /* m(j) = m_fine or m_fine 2^(J-j), Section 3.2 */
enum { BMG_SMOOTHER_MULTIPLICATIVE = 0, BMG_SMOOTHER_ADDITIVE = 1 };
enum { BMG_KAPPA_ARITHMETIC = 0, BMG_KAPPA_HARMONIC = 1 /* 0 if a child is 0 */, BMG_KAPPA_GEOMETRIC = 2 };
enum { BMG_COLOURING_S9 = 0,  /* 9 colours, (vx mod 3) + 3 (vy mod 3); a smoothing step is colours 0..8, 7..0 */
       BMG_COLOURING_L8 = 1   /* 8 colours, the cosets of the lattice spanned by (2, 2) and (2, -2):
                                 (vx mod 2) + 2 (vy mod 2) + 4 [(vx - vy) mod 4 >= 2]; colours 0..7, 6..0 */
};

typedef struct {
  int32_t n0;            /* cells per side of the coarsest mesh T_0, 2 <= n0 <= 64, and the coarsest
                            level has at most 4096 unknowns (its dense inverse is formed at setup):
                            n0 <= 36 (RT_0), 18 (RT_1), 12 (RT_2); BMG_E_UNSUPPORTED above that */
  int32_t levels;        /* J >= 0 refinements; finest N = n0 << levels <= 4096 */
  int32_t k;             /* Raviart-Thomas degree, 0, 1 or 2 (RT_k x dQ_k; Section 2) */
  double mu;             /* viscosity, >= 0 (0 = Darcy) */
  double sigma;          /* penalty constant; Section 4.1 uses (k+1)(k+2); face penalty 2 mu sigma / h_j */
  int32_t bc[4];         /* BMG_BC_* per side */
  int32_t cycle;         /* BMG_CYCLE_* */
  int32_t m_fine;        /* smoothing steps on the finest level, >= 1 (Section 4.1: 2) */
  int32_t precond_prec;  /* BMG_P_*: arithmetic of the V-cycle; the outer Krylov loop is always FP64 */
  int32_t restart;       /* FGMRES restart length, 1..512 */
  int32_t dense_coarse_max; /* 0..65535: the finest level jc >= 1 with at most this many dofs has its whole
                               sub-cycle B_jc (the same linear operator, Section 3.2) precomputed at setup
                               and applied as one dense matrix-vector product; 0 = none */
  int32_t n_rhs;         /* right-hand sides solved together, 1..16 (0 is read as 1).  Every vector
                            argument of a handle call then holds n_rhs columns of the level's ndof
                            entries, column r at offset r * ndof (column-major, contiguous) */
  int32_t colouring;     /* BMG_COLOURING_*: vertex colouring of the multiplicative smoother (the
                            order of the patch projections of Section 3.3; same-colour patches never
                            touch each other's dofs, so a colour is one parallel step) */
  int32_t smoother;      /* BMG_SMOOTHER_*: 0 (default) the symmetric multiplicative smoother of
                            eq. (smoother-Multiplicative); 1 the additive Schwarz smoother over the same
                            patch spaces, x += omega sum_v R_v^T A_v^+ R_v (b - A x) */
  double omega;          /* damping of the additive smoother, 0 < omega <= 1 (each cell lies in at
                            most four patches, so omega <= 1/4 keeps a step a contraction; 0.25 is
                            used in the tests); ignored by the multiplicative one */
  int32_t coarse_kappa;  /* BMG_KAPPA_*: kappa of a coarse cell from its four children; Section 4.1
                            uses the arithmetic mean (default) and notes that other choices are possible */
  int32_t setup_on_host; /* 0 (default): the patch pseudo-inverses are computed on the device (FP64
                            Gauss-Jordan, one workgroup per patch); 1: on the host (FP64 Gauss-Jordan on
                            every host thread).  The same matrices up to rounding */
  /* Tile parameters (performance only: the same method and results up to rounding; set
     by bmg_autotune_tiles, 0 = the built-in choice): */
  int32_t rotated_min_n;  /* one-column and FP64 handles: levels with at least this many cells per
                             side store their patch pseudo-inverses as rotated symmetric blocks
                             (about half the bytes, staged through LDS), smaller levels as full
                             blocks; 0 = 192; 0..4096 */
  int32_t columns_per_block; /* several-column handles on levels without the several-column
                                bfloat16 kernel: columns one block of the colour kernel applies a
                                patch inverse to; 0 = automatic; 0..16 */
} bmg_params;

typedef struct {
  int32_t iterations;            /* FGMRES iterations (preconditioner applications) */
  int32_t converged;             /* 1 if the residual estimate reached rtol */
  double rel_residual_estimate;  /* Arnoldi estimate / ||b|| at exit */
  double rel_residual_true;      /* ||b - A x|| / ||b|| recomputed in FP64 at exit */
} bmg_solve_info;

/* Device memory the library needs for these parameters (bmg_setup workspace). */
bmg_status bmg_plan(const bmg_params* p, size_t* workspace_bytes);

/* Build the hierarchy and every setup product: coarse kappa by averaging (p->coarse_kappa)
 * of the four children (Section 4.1), level operators, patch pseudo-inverses
 * (Section 3.3: the local Ritz projection on the vertex patch, pseudo-inverse with
 * zero patch-mean pressure when the patch problem has the constant-pressure null
 * mode), transfers and the coarse inverse (Section 3.2, B_0 = A_0^{-1}).
 *   kappa_host: N*N doubles, cell (cx, cy) at cy*N + cx, N = n0 << levels; finite,
 *               >= 0 if mu > 0 (0: Stokes), > 0 if mu = 0 (BMG_E_NONFINITE /
 *               BMG_E_ARG otherwise); copied, not retained.
 *   workspace_dev / bytes: caller-owned device memory of at least bmg_plan bytes
 *               (256-byte aligned), or NULL / 0 to let the library allocate it.
 *   hip_stream: hipStream_t for all work (NULL = default stream).
 *   out:        receives the handle. */
bmg_status bmg_setup(const bmg_params* p, const double* kappa_host, void* workspace_dev, size_t bytes,
                     void* hip_stream, bmg_handle* out);
/* Wait for the handle's stream, release its events, graph and capture stream, free
 * the workspace if the library allocated it (a caller-supplied workspace stays the
 * caller's), and delete the handle.  BMG_E_ARG for NULL. */
bmg_status bmg_destroy(bmg_handle h);

/* Sizes of level j (0 = coarsest, levels = finest). */
bmg_status bmg_sizes(bmg_handle h, int32_t level, int32_t* N, int64_t* n_u, int64_t* n_p);

/* y = A_j x, the saddle-point operator of level j (eq. Brinkman-weak) in FP64;
 * rows of the essential (constrained) normal dofs are the identity.  n_rhs columns. */
bmg_status bmg_apply(bmg_handle h, int32_t level, const double* x_dev, double* y_dev);

/* z = B_J r: one V-cycle (Section 3.2) in the handle's preconditioner arithmetic,
 * FP64 in and out, canonical layout of the finest level, n_rhs columns. */
bmg_status bmg_vcycle(bmg_handle h, const double* r_dev, double* z_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): z = B_J r as bmg_vcycle, with
 * the same kernels launched one by one on the handle's stream (no graph), and the
 * level vectors of the cycle (x_j, b_j, r_j of every level, n_rhs columns) kept
 * in a static device array of 256 MiB instead of the handle's workspace.  The
 * array exists once per device, from the library's load until the process ends,
 * and is shared by every handle on that device: calls that overlap on one device
 * (other streams, other threads) race on it.  Every level vector is written
 * before it is read, so nothing from an earlier call is used.  The call itself
 * allocates nothing (no hipMalloc, hipFree or graph); the first call on a device
 * looks up the array's device address (hipGetSymbolAddress).  BMG_E_NOMEM (with a
 * message) if 3 * sum_j ndof_j * w * (8 for BMG_P_FP64, else 4) bytes exceed 256 MiB,
 * where w = n_rhs, or for BMG_P_BF16 handles with n_rhs >= 2 and k >= 1 (whose level
 * vectors are interleaved records) n_rhs rounded up to a power of two >= 4. */
bmg_status bmg_vcycle_noalloc(bmg_handle h, const double* r_dev, double* z_dev);

/* Solve A_J x = b by right-preconditioned flexible GMRES(restart) in FP64 with B_J
 * as preconditioner (Section 3.2), until ||b - A x||_2 <= rtol ||b||_2 (Section 4.1
 * stopping rule with rtol as given).  A cycle ends when the Arnoldi estimate reaches
 * rtol; the next cycle starts from the true residual, which decides convergence
 * (iterative refinement); a cycle that reduces the true residual by less than 10%
 * ends the solve with BMG_E_NOT_CONVERGED (attainable accuracy reached).
 * With n_rhs > 1 every right-hand side runs its own FGMRES (own Krylov basis,
 * Hessenberg matrix, stopping test and iteration count); the iterations advance in
 * lockstep so that one V-cycle launch serves all columns, and a column that has
 * stopped is carried as zeros.  Column r gives the same iterates as a solve of b_r
 * alone.
 *   b_dev: the algebraic right-hand sides (n_rhs columns of n_u + n_p doubles,
 *          canonical layout), e.g. from bmg_assemble_rhs; x_dev: the solutions;
 *          x0_dev: initial guesses or NULL for zero.  Returns BMG_E_NOT_CONVERGED
 *          (with the last iterates) if some column did not reach rtol within maxit
 *          iterations; info: NULL or an array of n_rhs records, one per column. */
bmg_status bmg_solve(bmg_handle h, const double* b_dev, double* x_dev, double rtol, int32_t maxit,
                     const double* x0_dev, bmg_solve_info* info);

/* ----- batches of independent problems ----- */
/* Set up nprob independent problems (their own mesh, degree, mu, kappa, boundary
 * conditions and precision; params[i] and kappa_host[i] as for bmg_setup) that
 * are solved together.  The library allocates every problem's workspace and
 * nstreams worker streams (0 = 4, at most 16, default priority); the solves of a
 * batch call are spread over the worker streams, one host thread per stream, so
 * the V-cycles of different problems run concurrently on the GPU.  hip_stream is
 * the caller's stream that a batch call is ordered with (NULL = default stream).
 * Setup runs problem after problem (each uses every host thread). */
bmg_status bmg_batch_setup(int32_t nprob, const bmg_params* params, const double* const* kappa_host,
                           int32_t nstreams, void* hip_stream, bmg_batch_handle* out);
/* Solve every problem of the batch: b_dev[i] / x_dev[i] are device pointers (host
 * arrays of nprob pointers) laid out as for bmg_solve of problem i; info is NULL or
 * an array with one record per right-hand side of every problem, in problem order.
 * Work queued on the caller's stream before the call is waited for, and the
 * caller's stream waits for the batch.  Returns the first hard failure in problem
 * order, else BMG_E_NOT_CONVERGED if some problem did not converge, else BMG_OK;
 * bmg_batch_last_error names the problem. */
bmg_status bmg_batch_solve(bmg_batch_handle b, const double* const* b_dev, double* const* x_dev, double rtol,
                           int32_t maxit, bmg_solve_info* info);
/* The handle of problem i (sizes, single V-cycles, step entry points).  Owned by
 * the batch: do not destroy it, and do not use it while a batch call runs. */
bmg_status bmg_batch_handle_of(bmg_batch_handle b, int32_t i, bmg_handle* out);
/* Message of the last failing batch call (naming the problem). */
const char* bmg_batch_last_error(bmg_batch_handle b);
/* Wait for the worker streams, then free every problem's handle and workspace, the
 * worker streams and the batch.  BMG_E_ARG for NULL. */
bmg_status bmg_batch_destroy(bmg_batch_handle b);

/* ----- autotuning ----- */
/* Pick the smoother schedule for p: set up a handle for every candidate colouring
 * (S9, L8), time `trials` preconditioner applications (V-cycles, graph replay) on
 * hip_stream with HIP events, and write the parameters of the fastest into *best
 * (p with its colouring replaced).  ms_per_vcycle: NULL or 2 doubles, the measured
 * time per V-cycle of S9 and L8.  The candidates give the same method with another
 * order of the patch projections (Section 3.3); iteration counts are not measured.
 * Allocates and frees its own device memory; costs two setups. */
bmg_status bmg_autotune(const bmg_params* p, const double* kappa_host, void* hip_stream, int32_t trials,
                        bmg_params* best, double* ms_per_vcycle);
/* Pick the colouring and the tile parameters (rotated_min_n, columns_per_block) for p by
 * coordinate descent: the colourings first, then the storage threshold (192, 64, 4096),
 * then, for several columns outside the several-column bfloat16 kernel, the columns per
 * block (automatic, 1, 4, 16); every candidate is one setup timed over `trials` V-cycles
 * (graph replay, HIP events) on hip_stream.  The result is kept for the process, keyed
 * by (k, finest N, levels, precision, n_rhs, smoother, cycle, dense_coarse_max): a later
 * call with the same key returns it without timing (*n_report = 0).  report: NULL or
 * room for 4 * max_report doubles, one (colouring, rotated_min_n, columns_per_block,
 * ms per V-cycle) row per timed candidate; *n_report (may be NULL) the rows written.
 * Allocates and frees its own device memory. */
bmg_status bmg_autotune_tiles(const bmg_params* p, const double* kappa_host, void* hip_stream, int32_t trials,
                              bmg_params* best, double* report, int32_t max_report, int32_t* n_report);

/* ----- setup-side host calls (no handle, no device) ----- */
/* Quadrature points of bmg_assemble_rhs on the finest mesh of p (host arrays).
 * cell_xy: N*N cells x q*q points (point iy*q + ix) x 2, q = k+2 Gauss points per
 * direction; face_xy: 4 sides x N faces (ordered along the side) x q points x 2. */
bmg_status bmg_quad_points(const bmg_params* p, double* cell_xy_host, double* face_xy_host);

/* Right-hand side of eq. (BCh) on the finest mesh of p, FP64, host arrays:
 *   f_qp: source f at the cell points (x 2 components);
 *   s_qp: divergence source s (pressure rows -(s, q)) at the cell points, or NULL;
 *   g_qp: boundary data g at the face points (x 2), or NULL for g = 0; only
 *         Dirichlet sides are read; the normal component must be zero there
 *         (BMG_E_UNSUPPORTED otherwise), the tangential one enters through
 *         2 mu sigma_h <g, v> - mu <grad v n, g>.
 * Writes b (n_u + n_p doubles, canonical layout) to b_host. */
bmg_status bmg_assemble_rhs(const bmg_params* p, const double* f_qp, const double* s_qp, const double* g_qp,
                            double* b_host);

/* Vertex patch (vx, vy) of level 1 <= j <= levels (Section 3.3, the cells sharing
 * the vertex; dofs whose support lies in them, essential dofs excluded): writes n,
 * the dofs in ascending global order, its colour under p->colouring and, if
 * inv_host is not NULL, the FP64 pseudo-inverse of the patch matrix (row-major
 * n x n) exactly as setup computes it.  dofs_host must hold 12(k+1) + 8k(k+1) +
 * 4(k+1)^2 ints (an upper bound on n), inv_host the square of that many doubles.
 * kappa_host is the finest-level field as for bmg_setup. */
bmg_status bmg_export_patch(const bmg_params* p, const double* kappa_host, int32_t level, int32_t vx, int32_t vy,
                            int32_t* n, int32_t* dofs_host, double* inv_host, int32_t* colour);

/* Colour of every vertex (vx, vy) of level 1 <= j <= levels under p->colouring,
 * at vy * (N_j + 1) + vx of colour_host ((N_j + 1)^2 ints, may be NULL), and the
 * number of colours.  Patch p of a colour is the p-th vertex of that colour in
 * row-major order. */
bmg_status bmg_export_colouring(const bmg_params* p, int32_t level, int32_t* ncolours, int32_t* colour_host);

/* Dense A_j (row-major, FP64) of a level with at most 32 cells per side, from the
 * reference-element blocks the kernels use; essential rows/cols are the identity. */
bmg_status bmg_export_level_matrix(const bmg_params* p, const double* kappa_host, int32_t level, double* out_host);

/* ----- single steps of the cycle, for step-by-step checks (FP64 in/out, n_rhs
 * columns of the level's ndof entries) ----- */
/* One colour step of the multiplicative smoother on level j >= 1: for every vertex
 * patch of the colour (under p->colouring), x[S] += A_S^+ (b - A_j x)[S] (the same
 * step whatever p->smoother says). */
bmg_status bmg_colour_step(bmg_handle h, int32_t level, int32_t colour, double* x_dev, const double* b_dev);
/* `steps` applications of the smoother R_j of p->smoother (multiplicative: colours
 * 0..C-1 then C-2..0; additive: the damped sum of all patch corrections). */
bmg_status bmg_smooth(bmg_handle h, int32_t level, int32_t steps, double* x_dev, const double* b_dev);
/* b_{j-1} = P_j^T r_j (restriction; eq. 3 applied to residuals). */
bmg_status bmg_restrict(bmg_handle h, int32_t level, const double* rf_dev, double* bc_dev);
/* x_j += P_j z_{j-1} (natural injection of Section 3.1). */
bmg_status bmg_prolong_add(bmg_handle h, int32_t level, const double* xc_dev, double* xf_dev);
/* x_0 = A_0^{-1} b_0 (pseudo-inverse with zero mean pressure if A_0 is singular). */
bmg_status bmg_coarse_solve(bmg_handle h, const double* b_dev, double* x_dev);

/* ----- measurement ----- */
/* Record HIP events around the colour launches of the smoother on `level` (>= 1),
 * for at most max_launches launches from now on (-1 switches timing off).  One
 * event pair brackets the 2C - 1 back-to-back launches of each smoothing step (so
 * the timed span holds the short gaps between them); the events are recorded on
 * the handle's stream, and V-cycles run without the graph while timing is on. */
bmg_status bmg_kernel_timing(bmg_handle h, int32_t level, int32_t max_launches);
/* Launches timed so far, the summed duration of the bracketed spans and the bytes
 * the launches had to move (stored patch pseudo-inverses + gathered and scattered
 * vector entries). */
bmg_status bmg_kernel_timing_read(bmg_handle h, int32_t* launches, double* total_ms, double* bytes);

const char* bmg_status_string(bmg_status s);
/* Message of the last failure on h; with h == NULL, of the last bmg_setup or
 * bmg_batch_setup of the calling thread that failed after argument validation. */
const char* bmg_last_error(bmg_handle h);

#ifdef __cplusplus
}
#endif
#endif /* BMG_H */
