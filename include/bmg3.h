/*
 * bmg3.h -- C ABI of the 3-D (hexahedral) path of the MI355X geometric-multigrid
 * solver (Kanschat, Lazarov, Mao, arXiv 1602.04858).
 *
 * Problem (Section 2, d = 3): -mu Lap u + kappa u + grad p = f, div u = 0 on the unit
 * cube, mu >= 0 (mu = 0: the Darcy limit, eq. (Darcy-weak)), kappa >= 0 cellwise
 * constant; on a Dirichlet side u = g (for mu = 0 only the normal component counts),
 * on an open side the natural condition mu d_n u - p n = 0 (no boundary term, g not
 * used there; for mu = 0: p = 0).
 * Discretisation (Section 2): RT_k velocity x discontinuous Q_k pressure, k = 0 (the
 * lowest order, Section 2.3: one normal-flux dof per face, one pressure per cell) or
 * k = 1, on a uniform
 * N x N x N hexahedral mesh, interior-penalty form a_h (eq. ipbrinkman) with face
 * penalty 2 mu sigma / h, saddle-point form (eq. Brinkman-weak).  The normal velocity
 * on the boundary is an essential condition (boundary normal face dofs fixed, identity
 * rows), the tangential one is imposed by the Nitsche terms of eq. (BCh); with every
 * side Dirichlet the pressure is determined up to a constant (solutions are returned
 * as computed; compare pressures after removing the mean), an open side fixes it.
 * Solver (Section 3): FGMRES preconditioned by the V-cycle over N_j = n0 2^j with the
 * symmetric multiplicative vertex-patch smoother over patches of up to eight cells
 * (27 colours (vx mod 3) + 3 (vy mod 3) + 9 (vz mod 3), order 0..26, 25..0), the exact
 * embedding as prolongation, its transpose as restriction, and a dense solve on the
 * coarsest mesh.  Level operators, transfers and patch pseudo-inverses are assembled
 * on the host at setup; every step of a solve runs in the library's HIP kernels.
 *
 * Vector layout, with nb = k + 1, cell c = (cz N + cy) N + cx, velocity component d with
 * transverse axes (d1, d2) = the other two in increasing order, basis
 * psi_a(xi_d) L_b(xi_d1) L_c(xi_d2) (L_b orthonormal Legendre on [0,1], psi_0 = 1 - t,
 * psi_1 = t, psi_2 = int_0^t L_1) and pressure L_a(x) L_b(y) L_c(z):
 *   face dofs (a = 0/1, face index i = c_d + a along d):
 *       d NF + ((t2 N + t1)(N + 1) + i) nb^2 + b + nb c,   NF = (N + 1) N^2 nb^2
 *   interior dofs (a = 2, k = 1 only):  3 NF + c NI + d nb^2 + b + nb c,  NI = 3 k nb^2
 *   pressure:               n_u + c nb^3 + a + nb b + nb^2 c
 * with n_u = 3 NF + NI N^3 and n_p = nb^3 N^3; a full vector is velocity then pressure.
 *
 * Conventions: *_dev are device pointers owned by the caller, *_host host pointers;
 * device work runs on the stream given to bmg3_setup; a handle owns its device memory
 * (allocated in bmg3_setup, freed in bmg3_destroy) and is used by one host thread at a
 * time; every call returns a bmg_status and changes nothing on an argument error.
 */
#ifndef BMG3_H
#define BMG3_H

#include <stddef.h>
#include <stdint.h>

#include "bmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmg3_ctx* bmg3_handle;

typedef struct {
  int32_t n0;      /* coarsest mesh n0^3 cells, 1 .. 8 */
  int32_t levels;  /* >= 1; finest N = n0 2^(levels-1) <= 64 (RT_1), <= 128 (RT_0) */
  int32_t k;       /* RT degree: 0 or 1 */
  double mu;       /* viscosity >= 0 (0: Darcy) */
  double sigma;    /* penalty parameter > 0 (sigma_h = sigma / h); Section 4.1 uses (k+1)(k+2) */
  int32_t cycle;   /* 0: m_fine smoothing steps on every level; 1: variable, m_fine 2^(J-j) */
  int32_t m_fine;  /* >= 1 */
  int32_t restart; /* FGMRES restart length, 1 .. 200 */
  int32_t precond_prec; /* storage of the patch pseudo-inverses: 0 FP64, 1 FP32 (rounded to nearest;
                           vectors, residuals and arithmetic stay FP64; FGMRES absorbs the
                           perturbed V-cycle, as with the reduced-precision V-cycles of bmg.h) */
  int32_t bc[6];   /* BMG_BC_DIRICHLET / BMG_BC_OPEN per side: 0 x=0, 1 x=1, 2 y=0, 3 y=1, 4 z=0, 5 z=1 */
} bmg3_params;

/* Assemble levels, transfers and patch pseudo-inverses for the fine-level kappa
 * (kappa_host[c], N^3 values >= 0, finite; coarse kappa = mean of the eight children)
 * and upload them.  hip_stream: the hipStream_t every later call uses (NULL = default).
 * Cost at N = 32: ~17 s of host time and ~8 GB of device memory (6 GB of patch
 * pseudo-inverses: FP64 storage keeps the n (n/2 + 1) rotated diagonals of each
 * symmetric block, FP32 storage the full n x n block, about the same bytes); both
 * grow 8x per refinement, so N = 64 needs ~65 GB of device and host memory.
 * BMG_E_ARG on invalid parameters or kappa, BMG_E_NOMEM / BMG_E_HIP on device errors,
 * BMG_E_SINGULAR if a patch or the coarse matrix cannot be inverted. */
bmg_status bmg3_setup(const bmg3_params* p, const double* kappa_host, void* hip_stream, bmg3_handle* out);
/* Wait for the handle's stream, free its device memory and delete it.  BMG_E_ARG for NULL. */
bmg_status bmg3_destroy(bmg3_handle h);

/* Sizes of level `level` (0 = coarsest .. levels-1): cells per side, velocity and
 * pressure dofs, number of vertex patches ((N+1)^3). */
bmg_status bmg3_sizes(bmg3_handle h, int32_t level, int32_t* N, int64_t* n_u, int64_t* n_p, int64_t* npatch);

/* Right-hand side of eq. (BCh) on the finest level for constant body force f[3] and
 * constant boundary data g[3] (host array of n_u + n_p doubles): (f, v) + Nitsche
 * terms of g on the free rows minus the lifting of the essential values, the face
 * projection of g.n on the essential rows. */
bmg_status bmg3_assemble_rhs(const bmg3_params* p, const double* kappa_host, const double* f, const double* g,
                             double* b_host);

/* y = A_j x (level operator with identity essential rows); vectors of ndof(level). */
bmg_status bmg3_apply(bmg3_handle h, int32_t level, const double* x_dev, double* y_dev);
/* `steps` symmetric smoothing steps on level >= 1: x updated in place, b unchanged. */
bmg_status bmg3_smooth(bmg3_handle h, int32_t level, int32_t steps, double* x_dev, const double* b_dev);
/* z = B_J r: one V-cycle on the finest level (r unchanged). */
bmg_status bmg3_vcycle(bmg3_handle h, const double* r_dev, double* z_dev);
/* Solve A x = b with FGMRES(restart) and the V-cycle, x0 = 0, until the Arnoldi
 * residual estimate <= rtol ||b|| (then refined on the true residual as in bmg_solve)
 * or maxit preconditioner applications; BMG_E_NOT_CONVERGED with x the last iterate
 * otherwise.  BMG_E_NONFINITE if b holds a NaN or Inf (x untouched) or the iteration
 * produces one.  info may be NULL. */
bmg_status bmg3_solve(bmg3_handle h, const double* b_dev, double* x_dev, double rtol, int32_t maxit,
                      bmg_solve_info* info);
/* Dofs (ascending, *n of them, at most 256) and pseudo-inverse (n x n, column-major,
 * symmetrised: the mean of the computed inverse and its transpose, as the smoother
 * applies it) of the patch of vertex (vx, vy, vz) on level >= 1 (host arrays;
 * pinv_host may be NULL). */
bmg_status bmg3_export_patch(bmg3_handle h, int32_t level, int32_t vx, int32_t vy, int32_t vz, int32_t* n,
                             int32_t* dofs_host, double* pinv_host);
/* Host-only exports (no device needed) for checking the setup against a reference:
 * the CSR matrix of level `level` (call first with rp_host = NULL to get *nnz; then
 * rp_host holds ndof + 1 entries, ci_host and v_host *nnz), and the dofs and
 * symmetrised pseudo-inverse (column-major) of one vertex patch on level >= 1. */
bmg_status bmg3_export_level_csr(const bmg3_params* p, const double* kappa_host, int32_t level, int64_t* nnz,
                                 int32_t* rp_host, int32_t* ci_host, double* v_host);
bmg_status bmg3_export_patch_host(const bmg3_params* p, const double* kappa_host, int32_t level, int32_t vx,
                                  int32_t vy, int32_t vz, int32_t* n, int32_t* dofs_host, double* pinv_host);
/* Message of the last failing call on h (h = NULL: the last failed bmg3_setup). */
const char* bmg3_last_error(bmg3_handle h);

#ifdef __cplusplus
}
#endif

#endif /* BMG3_H */
