/*
 * sparc_filter.h -- C ABI of the MI355X Chebyshev-filter library.
 *
 * The library applies the discrete Kohn-Sham Hamiltonian of a real-space,
 * finite-difference isolated-cluster calculation and the Chebyshev polynomial
 * filter of the filtered subspace iteration built on it, following Ghosh &
 * Suryanarayana, "SPARC ... Part I: Isolated clusters" (arXiv:1603.04334):
 *
 *   H = -1/2 lap_h + diag(V_eff) + V_nl                         (Sec. 2, Eq. EL)
 *   lap_h f = sum_{p=0..n_o} w_p (six values at distance p)     (Sec. 3.1, Eq. FD:Laplacian)
 *   w_p as in Sec. 3.1 Eq. weightsLap; f = 0 off the grid      (zero Dirichlet, Sec. 3.1)
 *   V_nl f = h^3 sum_J sum_lm gamma_Jl chi_Jlm chi_Jlm^T f      (Sec. 3.1, Eq. non-localPS:FD)
 *   Psi_f = p_m(H) Psi,  p_m(t) = C_m((t - c)/e)                (Sec. 3.4, Eq. ChebFilter, Alg. 2)
 *   H_s = Psi_f^T H Psi_f, M_s = Psi_f^T Psi_f, H_s y = l M_s y (Sec. 3.4, Eq. SubspaceGeneralizedEigenproblem)
 *   Psi = Psi_f Y                                               (Sec. 3.4, Eq. OrbitalTransformation)
 *
 * Conventions shared by every call:
 *   - Grid: n[0] x n[1] x n[2] nodes (x, y, z); linear node index
 *     k + n[2]*(j + n[1]*i), z fastest.  N_d = n[0]*n[1]*n[2].
 *   - Orbital blocks are dense N_d x ns matrices in column-major order (the
 *     orbitals are the columns, Sec. 3.1): column c starts at element c*ld,
 *     ld >= N_d.  They live in device memory owned by the caller.
 *   - dtype selects the storage and arithmetic type of an orbital block:
 *     SPARC_F64 (double) or SPARC_F32 (float, FP32 accumulation; filter
 *     coefficients are computed in FP64 and rounded once).
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it and the call returns; results are valid once the
 *     stream has reached that point.  Calls documented as synchronous wait.
 *   - Workspace: calls that need scratch memory take a caller-owned device
 *     buffer ws of at least the size returned by the matching *_bytes query.
 *     Concurrent calls need distinct workspaces.
 *   - Units are Hartree and bohr.
 *   - Every call returns a sparc_status; on failure nothing has been enqueued
 *     and sparc_last_error() gives a message for the calling thread.
 */
#ifndef SPARC_FILTER_H
#define SPARC_FILTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPARC_OK = 0,
    SPARC_PENDING = 1,       /* job not finished (poll)                          */
    SPARC_E_ARG = -1,        /* null pointer, bad enum, bad count                */
    SPARC_E_SHAPE = -2,      /* grid / box / leading dimension inconsistent      */
    SPARC_E_BOUNDS = -3,     /* filter bounds not a0 < a < b, or m < 1           */
    SPARC_E_NOMEM = -4,      /* device allocation failed / budget exceeded       */
    SPARC_E_HIP = -5,        /* a HIP runtime or library call failed             */
    SPARC_E_BUSY = -6,       /* reserved                                         */
    SPARC_E_TICKET = -7,     /* unknown ticket                                   */
    SPARC_E_JOB = -8,        /* job failed (see sparc_job_result.status)         */
    SPARC_E_WORKSPACE = -9,  /* workspace missing or too small                   */
    SPARC_E_BREAKDOWN = -10, /* Lanczos invariant subspace / singular M_s        */
    SPARC_E_ALIAS = -11      /* input and output / workspace overlap             */
} sparc_status;

typedef enum { SPARC_F64 = 0, SPARC_F32 = 1 } sparc_dtype;

/* Uniform finite-difference grid of Sec. 3.1: n nodes per axis, spacing h,
 * stencil half-width radius = n_o (1..6; the paper uses 6). */
typedef struct {
    int32_t n[3];
    double h;
    int32_t radius;
} sparc_grid;

/* One atom's Kleinman-Bylander projectors (Sec. 2 Eq. V_nl, Sec. 3.1 Eq.
 * non-localPS:FD), restricted to a cube of nodes (Sec. 3.2 uses cubes around
 * atoms).  lo: first node index of the cube per axis (0-based); ext: cube
 * extent per axis; the cube must lie inside the grid.  chi: host array of
 * nproj*ext[0]*ext[1]*ext[2] values, projector slowest then x, y, z fastest;
 * the h^3 quadrature weight is NOT folded in.  gamma: host array of nproj
 * projector energies (gamma_Jl repeated over m).  1 <= nproj <= 16.  Both
 * arrays are copied by sparc_op_create. */
typedef struct {
    int32_t lo[3];
    int32_t ext[3];
    int32_t nproj;
    const double *chi;
    const double *gamma;
} sparc_atom;

typedef struct sparc_op sparc_op;

/* ------------------------------------------------------------------ operator */

/* Build the discrete Hamiltonian of one cluster on the current HIP device.
 * veff: host array of N_d values of V_eff at the nodes.  The op keeps device
 * copies of V_eff and chi in FP64 and FP32 and the index tables of the
 * projector cubes, and nothing else; it may be used from several streams at
 * once (sparc_op_set_launch aside).  Synchronous.
 * Errors: SPARC_E_ARG (null pointers, natoms < 0, nproj outside 1..16),
 * SPARC_E_SHAPE (n < 1, n[1]*n[2] >= 2^28, h <= 0, radius outside 1..6,
 * cube outside the grid),
 * SPARC_E_NOMEM, SPARC_E_HIP. */
int sparc_op_create(const sparc_grid *grid, const double *veff, int32_t natoms,
                    const sparc_atom *atoms, sparc_op **out);

/* Release the op's device memory.  The caller must make sure no enqueued work
 * still uses it.  NULL is accepted. */
int sparc_op_destroy(sparc_op *op);

/* N_d of the op's grid, and the total number of projectors. */
int64_t sparc_op_nd(const sparc_op *op);
int32_t sparc_op_nproj(const sparc_op *op);

/* Workspace in bytes needed by sparc_h_apply (which = 0) or by
 * sparc_cheb_filter (which = 1) for ns columns of the given dtype. */
size_t sparc_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns, int32_t which);

/* Y = H X for ns columns (Sec. 2 Eq. EL operator discretised as in Sec. 3.1).
 * X (ldx) and Y (ldy) are device blocks of the given dtype and must not
 * overlap.  ws: device workspace of sparc_workspace_bytes(op, dtype, ns, 0)
 * bytes (may be NULL when the op has no atoms).  Asynchronous.
 * Errors: SPARC_E_ARG, SPARC_E_SHAPE (ld < N_d, ns < 1), SPARC_E_ALIAS,
 * SPARC_E_WORKSPACE, SPARC_E_HIP. */
int sparc_h_apply(const sparc_op *op, int32_t dtype, const void *X, int64_t ldx, void *Y, int64_t ldy,
                  int32_t ns, void *ws, size_t ws_bytes, void *stream);

/* Y = H X as sparc_h_apply, without allocation and without a workspace
 * argument: for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * projector gather partials live in a fixed device array of
 * sparc_noalloc_scratch_bytes() bytes (16 MiB) that every GPU the library
 * runs on holds until the process ends; the first call on a device looks up
 * its address.  Calls that need more (8 * nproj_total * ns * element size,
 * i.e. nproj_total * ns up to 262144 in FP64 or 524288 in FP32) fail with
 * SPARC_E_WORKSPACE.  Nothing in the array needs clearing between calls.
 * All calls on one GPU share the array: calls that overlap in time on one
 * GPU (on different streams or threads) race and must not be made.  Results
 * are bitwise those of sparc_h_apply.  Asynchronous.
 * Errors: as sparc_h_apply, SPARC_E_WORKSPACE (scratch too small). */
int sparc_h_apply_noalloc(const sparc_op *op, int32_t dtype, const void *X, int64_t ldx, void *Y, int64_t ldy,
                          int32_t ns, void *stream);

/* Size in bytes of the fixed scratch array of sparc_h_apply_noalloc. */
size_t sparc_noalloc_scratch_bytes(void);

/* Chebyshev filter of degree m (Sec. 3.4, Eq. ChebFilter and Alg. 2) in the
 * scaled three-term form of the filtered subspace iteration the paper cites:
 *   e = (b - a)/2, c = (b + a)/2, sigma_1 = e/(a0 - c), tau = 2/sigma_1,
 *   Y_1 = (sigma_1/e)(H - cI)X,
 *   Y_{k+1} = (2 sigma_{k+1}/e)(H - cI)Y_k - sigma_k sigma_{k+1} Y_{k-1},
 *   sigma_{k+1} = 1/(tau - sigma_k),  k = 1..m-1,
 * so Y = C_m((H - c)/e) X / C_m((a0 - c)/e): eigencomponents in [a, b] are
 * damped and the component at a0 passes with gain 1.
 * a0 plays lambda_1, a the cutoff lambda_c and b lambda_{N_d} of Alg. 2.
 * X (ldx) is read only; Y (ldy) receives the result; neither may overlap the
 * other or ws.  ws: sparc_workspace_bytes(op, dtype, ns, 1) bytes.
 * Asynchronous: 3m kernel launches (m when the op has no atoms).
 * Errors: SPARC_E_BOUNDS (m < 1 or not a0 < a < b), SPARC_E_ARG,
 * SPARC_E_SHAPE, SPARC_E_ALIAS, SPARC_E_WORKSPACE, SPARC_E_HIP. */
int sparc_cheb_filter(const sparc_op *op, int32_t dtype, const void *X, int64_t ldx, void *Y, int64_t ldy,
                      int32_t ns, int32_t m, double a0, double a, double b, void *ws, size_t ws_bytes,
                      void *stream);

/* --------------------------------------------------------- spectral bounds */

/* Workspace bytes of sparc_lanczos for k steps. */
size_t sparc_lanczos_workspace_bytes(const sparc_op *op, int32_t k);

/* k steps of Lanczos on H in FP64 on the device (Sec. 4: extremal eigenvalues
 * of H by a few Lanczos iterations), kept semi-orthogonal by partial
 * re-orthogonalisation: the loss of orthogonality is estimated on the device
 * from the coefficients (Simon's recurrence) and, whenever an estimate passes
 * sqrt(eps), that step and the next are orthogonalised against the whole basis
 * by classical Gram-Schmidt.  T_k then agrees with a fully re-orthogonalised
 * run to working accuracy.  v0: device FP64 start vector of N_d
 * values (normalised internally, not modified).  Outputs on the host: alpha[k]
 * and beta[k-1] (the tridiagonal T_k, may be NULL) and theta[k], the
 * eigenvalues of T_k in ascending order.  Synchronous (waits for stream).
 * Errors: SPARC_E_ARG (k < 1 or k > N_d), SPARC_E_WORKSPACE,
 * SPARC_E_BREAKDOWN (a beta_j vanished), SPARC_E_HIP. */
int sparc_lanczos(const sparc_op *op, int32_t k, const double *v0, double *alpha, double *beta,
                  double *theta, void *ws, size_t ws_bytes, void *stream);

/* Guaranteed upper bound on the largest eigenvalue of H: three times the
 * maximum of the 1D stencil symbol of -1/2 lap_h, plus max V_eff, plus
 * h^3 max(gamma_J,0) trace(chi_J^T chi_J) per atom.  Host only. */
int sparc_upper_bound(const sparc_op *op, double *ub);

/* Filter bounds from ascending Ritz values theta[k]: a0 = theta[0],
 * a = theta[nwant-1] + shift, b = bfactor*theta[k-1], and b is lowered to
 * ubound when ubound < b (pass ubound <= 0 to skip).
 * Errors: SPARC_E_ARG, SPARC_E_BOUNDS (result not a0 < a < b).  Host only. */
int sparc_select_bounds(const double *theta, int32_t k, int32_t nwant, double shift, double bfactor,
                        double ubound, double *a0, double *a, double *b);

/* ------------------------------------------------------- Rayleigh-Ritz step */

/* Workspace bytes of sparc_rayleigh_ritz for ns columns of the given dtype. */
size_t sparc_rr_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns);

/* Rayleigh-Ritz on the filtered block (Sec. 3.4): with Y promoted to FP64,
 * H_s = Y^T (H Y) and M_s = Y^T Y (the h^3 factors cancel), then the
 * symmetric-definite problem H_s q = theta M_s q, all in FP64 on the device.
 * theta: host array of ns Ritz values, ascending.  evec: optional device FP64
 * ns x ns column-major array receiving the M_s-orthonormal eigenvectors (the
 * rotation matrix of Eq. OrbitalTransformation).  Synchronous.
 * Errors: SPARC_E_ARG, SPARC_E_SHAPE (also 8 ldy + nd >= 2^32), SPARC_E_WORKSPACE,
 * SPARC_E_HIP, SPARC_E_BREAKDOWN (M_s not numerically positive definite: the
 * filtered columns are linearly dependent to working precision). */
int sparc_rayleigh_ritz(const sparc_op *op, int32_t dtype, const void *Y, int64_t ldy, int32_t ns,
                        double *theta, double *evec, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes of sparc_rotate: a zero-padded copy of Q in dtype. */
size_t sparc_rotate_workspace_bytes(int32_t dtype, int32_t ns);

/* Subspace rotation Psi = Psi_f Q (Sec. 3.4, Eq. OrbitalTransformation):
 * Y (ldy) is an nd x ns block of the given dtype, Q an FP64 ns x ns
 * column-major device matrix (rounded to dtype for an FP32 block), ws a device
 * workspace of sparc_rotate_workspace_bytes(dtype, ns) bytes, out (ldo) an
 * nd x ns block of dtype.  Sums run in dtype.  Blocks of up to 64 (FP32) /
 * 32 (FP64) columns take the library's kernel, which reads Y once; wider
 * blocks a rocBLAS GEMM (atomics off, so results are reproducible).  Y, out
 * and ws must not overlap.  Asynchronous.  Errors: SPARC_E_ARG,
 * SPARC_E_SHAPE, SPARC_E_WORKSPACE, SPARC_E_ALIAS, SPARC_E_HIP. */
int sparc_rotate(int32_t dtype, const void *Y, int64_t ldy, int64_t nd, int32_t ns, const double *Q,
                 void *out, int64_t ldo, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------- occupations and density */

/* Fermi energy (Sec. 3.4, Eq. FermiEnergyConstraintFormulation): the root
 * lambda_f of 2 sum_n g_n = N_e with g_n = 1 / (1 + exp((theta_n -
 * lambda_f) / kT)), found by Brent's method as in Sec. 4 (the paper's runs
 * use kT = 1e-3 Ha).  theta: host array of ns eigenvalues (any order); ne:
 * electron count, 0 < ne < 2 ns; kT > 0 in the units of theta.  lambda_f
 * receives the root, to about 1e-15 relative; occ, when not null, a host
 * array of ns occupations g_n.  The residual is evaluated without
 * cancellation, so the root is determined across gaps of up to about 1400 kT;
 * wider gaps leave a flat residual and any point of the gap is returned.
 * Errors: SPARC_E_ARG (null pointers, ns < 1, ne outside (0, 2 ns), kT <= 0,
 * non-finite theta), SPARC_E_BOUNDS (no bracket found).  Host only. */
int sparc_fermi_level(const double *theta, int32_t ns, double ne, double kT, double *lambda_f, double *occ);

/* Electron density on the grid (Sec. 3.4): rho[i] = (2/h^3) sum_n occ[n]
 * psi_n[i]^2 for the nd x ns block psi (column n = orbital n at psi + n ld,
 * dtype SPARC_F64 or SPARC_F32), occ a device FP64 array of ns occupations,
 * rho a device FP64 array of nd values (overwritten).  Products and sums run
 * in FP64, columns in ascending order, so the result is independent of the
 * launch.  One pass over psi: s nd ns bytes read, 8 nd written.  rho must not
 * overlap psi.  Asynchronous on stream.  Errors: SPARC_E_ARG, SPARC_E_SHAPE
 * (nd < 1, ld < nd, h <= 0), SPARC_E_ALIAS, SPARC_E_HIP. */
int sparc_density(int32_t dtype, const void *psi, int64_t ld, int64_t nd, int32_t ns, const double *occ, double h,
                  double *rho, void *stream);

/* ------------------------------------------------------- nonlocal force */

/* Workspace bytes of sparc_nonlocal_force for ns orbitals (0 on bad arguments). */
size_t sparc_force_workspace_bytes(const sparc_op *op, int32_t ns);

/* Nonlocal component of the atomic forces (Sec. 3.6, Eqs.
 * NonlocForce:Discrete and NonLocForce:U:W, Alg. 4):
 * f_J = -4 sum_n occ[n] sum_lm gamma_Jl Y_Jnlm W_Jnlm with
 * Y_Jnlm = h^3 sum psi_n chi_Jlm and W_Jnlm = h^3 sum (grad_h psi_n) chi_Jlm,
 * grad_h the finite-difference gradient of Eq. gradient:approximate (order
 * 2 n_o, the operator's stencil radius, zero Dirichlet padding).  psi: the
 * nd x ns block (column n at psi + n ld, dtype SPARC_F64 or SPARC_F32,
 * widened to FP64 as it is read); occ: device FP64 array of ns occupations;
 * force: device FP64 array of 3 natoms values, atom J's (x, y, z) at 3J
 * (overwritten); ws: device workspace of sparc_force_workspace_bytes bytes.
 * All sums run in FP64 in a fixed order.  The first call on an operator
 * builds its gradient tables (FP64, about 4x the projector data) and is
 * synchronous; later calls are asynchronous on stream.  With no atoms
 * nothing is written.  Errors: SPARC_E_ARG, SPARC_E_SHAPE,
 * SPARC_E_WORKSPACE, SPARC_E_ALIAS, SPARC_E_NOMEM, SPARC_E_HIP. */
int sparc_nonlocal_force(const sparc_op *op, int32_t dtype, const void *psi, int64_t ld, int32_t ns, const double *occ,
                         double *force, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------- electrostatic potential */

typedef struct sparc_poisson sparc_poisson;

/* A Poisson solver for the grid (n, h, stencil radius n_o as for
 * sparc_op_create): the operator -(1/4 pi) lap_h with zero Dirichlet padding
 * (Sec. 3.3, Eq. FD:PoissonDiscrete), the multipole boundary correction to
 * order lmax (0..6; the paper uses 6, Sec. 4), and the block-Jacobi
 * preconditioner on blocks of block[0] x block[1] x block[2] nodes (each edge
 * 1..8, at most 256 nodes; NULL = 4 x 4 x 4; blocks at the high end of an
 * axis are cut short), whose block inverses are formed here (host, FP64).
 * The expansion centre is the centre of the domain.  Allocates on the
 * current device.  Errors: SPARC_E_ARG, SPARC_E_SHAPE, SPARC_E_NOMEM,
 * SPARC_E_HIP. */
int sparc_poisson_create(const sparc_grid *grid, int32_t lmax, const int32_t *block, sparc_poisson **out);

/* Free the solver.  NULL is accepted. */
int sparc_poisson_destroy(sparc_poisson *p);

/* Workspace bytes of sparc_poisson_solve (four grid vectors, the boundary
 * slabs and the reduction partials). */
size_t sparc_poisson_workspace_bytes(const sparc_poisson *p);

/* Electrostatic potential of the total charge c = rho + b (Sec. 3.3):
 * -(1/4 pi) lap_h phi = c - d (Eq. FD:PoissonDiscrete), d the charge
 * correction of Eq. Phi:correction with phi off the grid from the multipole
 * expansion of Eq. phi:BC:discrete, moments Q_lm = h^3 sum |x|^l Y_lm c (real
 * orthonormal Y_lm).  Preconditioned CG from phi = 0 (use_guess = 0) or from
 * the values in phi (use_guess = 1) until ||r||_2 <= tol ||c - d||_2 (r the
 * recursively updated residual) or max_iter iterations.  charge, phi: device
 * FP64 arrays of N_d values (phi overwritten with the solution); iters,
 * rel_resid: host outputs (may be NULL); moments: NULL or a host array of
 * (lmax+1)^2 values receiving Q_lm (index l*l + l + m).  All sums FP64 in a
 * fixed order (reproducible bit for bit).  Synchronous on stream (it reads a
 * convergence flag every 8 iterations).  Errors: SPARC_E_ARG (tol <= 0,
 * max_iter < 0), SPARC_E_WORKSPACE, SPARC_E_ALIAS, SPARC_E_SHAPE, SPARC_E_HIP. */
int sparc_poisson_solve(sparc_poisson *p, const double *charge, double *phi, int32_t use_guess, double tol,
                        int32_t max_iter, int32_t *iters, double *rel_resid, double *moments, void *ws,
                        size_t ws_bytes, void *stream);

/* ------------------------------------------------------- CheFSI passes */

/* Workspace bytes of sparc_chefsi (0 on bad arguments). */
size_t sparc_chefsi_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns);

/* `passes` CheFSI passes on the orbital block X in place (Sec. 3.4): the
 * Chebyshev filter (bounds a0, lambda_c, b), the FP64 Rayleigh-Ritz step, the
 * Fermi level of the Ritz values (as sparc_fermi_level, with ne and kT) and
 * the subspace rotation, after which X holds the Ritz vectors.  The first
 * SCF iteration of a calculation runs about three passes from a random block
 * (Sec. 3.4, last paragraph), every later one a single pass.  The first pass
 * uses the cutoff a; every later pass the previous pass's Fermi level + 0.1 Ha
 * (Sec. 4).  b is fixed (H does not change between the passes); so is a0,
 * except that when a later cutoff falls at or below it (the Lanczos estimate
 * of lambda_1 had missed a low state) a0 becomes the lowest Ritz value of the
 * previous pass; a0 only scales the filter's output.  A caller chaining
 * calls applies the same rule with the theta it received.
 * A pass whose filtered block is numerically rank deficient (the Cholesky
 * factorisation of M_s fails) is filtered again from the same X at half the
 * degree, down to degree 1; degrees reports the degree each pass used.
 * X: device block of dtype, ns columns, leading dimension ldx; ws: device
 * workspace of sparc_chefsi_workspace_bytes bytes.  Host outputs (each may be
 * NULL): theta (passes x ns Ritz values, pass by pass, ascending), lambda_f
 * (passes Fermi levels), degrees (passes degrees).  rho: NULL, or a device
 * FP64 array of N_d values receiving the density of the final block with
 * the final occupations (as sparc_density).  Synchronous on stream.
 * Errors: SPARC_E_ARG (bad dtype, passes < 1, ne outside (0, 2 ns), kT <= 0),
 * SPARC_E_SHAPE, SPARC_E_BOUNDS (m < 1, not a0 < a < b, or a Fermi-level
 * cutoff outside (a0, b)), SPARC_E_WORKSPACE, SPARC_E_ALIAS, SPARC_E_HIP,
 * SPARC_E_BREAKDOWN (rank deficient at degree 1, or an eigensolver that did
 * not converge).  On error X may hold the rotated block of an earlier pass. */
int sparc_chefsi(const sparc_op *op, int32_t dtype, void *X, int64_t ldx, int32_t ns, int32_t m, int32_t passes,
                 double ne, double kT, double a0, double a, double b, double *theta, double *lambda_f,
                 int32_t *degrees, double *rho, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------- batched filters */

/* One filter of a batch: the arguments of sparc_cheb_filter for one cluster.
 * X and Y stay owned by the caller and must stay allocated while the batch
 * exists; the batch owns the workspaces. */
typedef struct {
    const sparc_op *op;
    int32_t dtype;
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    int32_t ns;
    int32_t m;
    double a0, a, b;
} sparc_batch_job;

typedef struct sparc_batch sparc_batch;

/* Build a batch of Chebyshev filters over uneven clusters (Sec. 3.4 applied
 * to each job).  Every filter is cut into the work items of its degree steps
 * (projector gather and stencil patches of step k, then the projector scatter
 * of step k), items are ordered level by level across the batch, and
 *   mode 0: one persistent launch takes items from an atomic ticket and waits
 *           per cluster for the items each depends on (device-scope
 *           release/acquire counters, bounded waits), captured together with
 *           the counter reset in a HIP graph that later runs replay;
 *   mode 1: the same persistent launch without the graph;
 *   mode 2: one grouped launch per level (no waits);
 *   mode 3: the plain filters one after another;
 *   mode 4: mode 2 captured in a HIP graph (replayed on later runs);
 *   mode 5: the plain filters on four streams owned by the batch (jobs dealt
 *           longest first to the least loaded one), started after the work
 *           already on `stream` and joined back to it by events; the
 *           filters of different jobs overlap.  Each job still runs on one
 *           stream with its own workspace.
 * Every mode gives each job exactly the result of sparc_cheb_filter.
 * Allocates the per-job workspaces and the schedule on the current device.
 * Errors: SPARC_E_ARG, SPARC_E_BOUNDS, SPARC_E_SHAPE, SPARC_E_NOMEM, SPARC_E_HIP. */
int sparc_batch_create(const sparc_batch_job *jobs, int32_t njobs, int32_t mode, sparc_batch **out);

/* Enqueue one run of the whole batch on stream.  Asynchronous. */
int sparc_batch_run(sparc_batch *batch, void *stream);

/* Wait for stream and report whether the last run aborted (a dependency wait
 * exceeded its bound; results are then invalid): SPARC_OK or SPARC_E_JOB. */
int sparc_batch_check(sparc_batch *batch, void *stream, int32_t *aborted);

/* Work items, levels and persistent grid size of a batch (out params may be NULL). */
int sparc_batch_info(const sparc_batch *batch, int64_t *items, int32_t *levels, int32_t *grid);

/* Free the batch (its graph, schedule and workspaces).  NULL is accepted. */
int sparc_batch_destroy(sparc_batch *batch);

/* ------------------------------------------------------------------ serving */

/* Server configuration: device memory budget for resident clusters (0 = 250 GB),
 * number of worker threads (requests on the device at once, each on its own
 * stream; 1..64), Lanczos steps for the bounds (0 = 40), CheFSI passes of a
 * cluster's first request (0 = 3, at most 64; Sec. 3.4, last paragraph) and
 * the smearing k_B T of the Fermi level (0 = 1e-3 Ha, Sec. 4). */
typedef struct {
    uint64_t hbm_budget_bytes;
    int32_t workers;
    int32_t lanczos_steps;
    int32_t first_passes;
    double kT;
} sparc_server_cfg;

/* A cluster: the operator (as for sparc_op_create), dtype, orbital count ns
 * and filter degree m, its initial orbitals X0 (device block of dtype, ns
 * columns, leading dimension ldx0), the device FP64 Lanczos start v0 (N_d
 * values) and its electron count ne (0 < ne < 2 ns; the paper sizes
 * ns = ne/2 + 30, Sec. 4).  Host arrays are copied at submission; X0 and v0 must be complete
 * (their producing work finished) when the first request is submitted, are
 * read when the cluster is admitted and must stay valid until that request is
 * done.  The server copies X0, so the caller's block is never written. */
typedef struct {
    sparc_grid grid;
    const double *veff;
    int32_t natoms;
    const sparc_atom *atoms;
    int32_t dtype;
    int32_t ns;
    int32_t m;
    const void *X0;
    int64_t ldx0;
    const double *v0;
    double ne;
} sparc_cluster_desc;

/* One request: the eigensolve of one SCF iteration on the resident orbitals
 * of cluster `cluster` (an id chosen by the caller), in the cluster's dtype
 * throughout.  The first request of a cluster carries its description; it
 * builds the operator, copies X0, computes the filter bounds with the device
 * Lanczos (a0 = theta_1, cutoff theta_8 + 0.1, b = 1.01 theta_max capped by
 * the upper bound) and runs the first-SCF rule: first_passes CheFSI passes
 * (as sparc_chefsi) from X0 without a density update (Sec. 3.4, last
 * paragraph).  Every later request runs one pass on the resident rotated
 * orbitals.  After the first pass every cutoff is the previous pass's Fermi
 * level + 0.1 Ha (Sec. 4), carried across requests; a0 and b are kept.
 * release = 1 frees the cluster's device memory after this request.  ritz:
 * optional host buffer of ns doubles receiving the Ritz values of the
 * request's last pass; it must stay valid until the request is done. */
typedef struct {
    uint64_t cluster;
    const sparc_cluster_desc *desc;
    int32_t release;
    double *ritz;
} sparc_filter_job;

/* Outcome of a request: status (SPARC_OK or the failing call's code;
 * SPARC_E_JOB when an earlier request of the cluster failed), 0-based index of
 * the request within its cluster, steady-clock times (seconds, as
 * sparc_clock) of submission, start and completion, lowest Ritz value and
 * Fermi level of the last pass, N_d * ns * (sum of the passes' degrees)
 * filtered orbital*gridpoint updates, the number of passes run and of degree
 * halvings (rank-deficient passes redone at half the degree). */
typedef struct {
    int32_t status;
    int32_t step;
    double t_submit, t_start, t_end;
    double lambda_min;
    int64_t updates;
    double lambda_f;
    int32_t passes;
    int32_t halvings;
    char error[128];  /* message of the failing call (empty on success) */
} sparc_job_result;

typedef struct sparc_server sparc_server;

/* Start a server on the current device with cfg->workers worker threads. */
int sparc_server_create(const sparc_server_cfg *cfg, sparc_server **out);

/* Queue a request; returns at once with a ticket.  A cluster is admitted when
 * its estimated device footprint fits the budget beside the resident
 * clusters; requests of one cluster run in submission order; requests of
 * different clusters run concurrently (continuous batching).
 * Errors: SPARC_E_ARG (bad or duplicate description, unknown cluster),
 * SPARC_E_BOUNDS, SPARC_E_SHAPE, SPARC_E_NOMEM (footprint above the whole
 * budget), SPARC_E_JOB (cluster already released or failed). */
int sparc_filter_submit(sparc_server *srv, const sparc_filter_job *job, uint64_t *ticket);

/* SPARC_OK with the result when the request is done (the ticket is then
 * retired), SPARC_PENDING while it waits or runs, SPARC_E_TICKET for an
 * unknown or retired ticket. */
int sparc_filter_poll(sparc_server *srv, uint64_t ticket, sparc_job_result *result);

/* Counts of finished (not yet polled or polled), pending and running requests,
 * and the reserved device bytes. */
int sparc_server_stats(sparc_server *srv, int64_t *done, int64_t *pending, int64_t *running, uint64_t *hbm_used);

/* Cluster records the server holds on the host (clusters submitted and not
 * yet released or failed, with their copies of V_eff and the projectors), and
 * the number of retired ids: a released or failed cluster's record is freed
 * once no queued request refers to it, and its id is refused from then on. */
int sparc_server_clusters(sparc_server *srv, int64_t *records, int64_t *retired);

/* Finish running requests, drop pending ones, free every cluster, stop the workers. */
int sparc_server_destroy(sparc_server *srv);

/* Seconds on the steady clock used for request times. */
double sparc_clock(void);

/* Device bytes the server reserves for a cluster when admitting it (operator,
 * resident orbitals, filter, Rayleigh-Ritz and Lanczos workspaces).  Host only. */
uint64_t sparc_cluster_footprint(const sparc_cluster_desc *desc, int32_t lanczos_steps);

/* ------------------------------------------------------------- diagnostics */

/* Plain device copy of `bytes` bytes (a multiple of 16, both addresses
 * 16-byte aligned, not overlapping), one 16-byte unit per lane with
 * non-temporal accesses: the reference bandwidth the step kernels are
 * compared with, and the known-size workload that calibrates the hardware
 * traffic counters.  Asynchronous on stream.
 * Errors: SPARC_E_ARG, SPARC_E_ALIAS, SPARC_E_SHAPE, SPARC_E_HIP. */
int sparc_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

const char *sparc_status_str(int status);
const char *sparc_last_error(void);

/* Number of times a rocSOLVER / rocBLAS call of the Rayleigh-Ritz eigensolver
 * returned success but left
 * the thread's HIP error state set to hipErrorStreamCaptureUnsupported, which
 * the library then cleared (each occurrence up to the eighth is also written
 * to stderr).  Any other error code left behind fails the call with
 * SPARC_E_HIP instead.  Host only. */
int64_t sparc_cleared_hip_errors(void);

/* Per-kernel timing with HIP events recorded around each launch on the
 * launching stream.  kernel: 0 = fused stencil/potential/recurrence step
 * with Y_{k-1} (k >= 1), 1 = projector gather, 2 = projector scatter, 3 = the
 * same fused step without Y_{k-1} (first filter step, H application), 4 =
 * the density pass, 5 = the nonlocal-force reduction, 6 = the Poisson
 * operator, 7 unused.  enable(1) starts recording;
 * read() synchronises the recorded events and returns the number of launches
 * and their summed duration in ms; reset() clears the counts. */
int sparc_profile_enable(int32_t on);
int sparc_profile_read(int32_t kernel, int64_t *launches, double *total_ms);
int sparc_profile_reset(void);

/* Override the launch configuration of the vector step kernels (the fused
 * stencil / potential / recurrence pass with the projections of its input
 * gathered in its last workgroups) for one dtype: patch extent along z and y
 * (FP32: tile_z = 32 with tile_y 16, 32 or 64; tile_z = 64 with tile_y 16 or
 * 32; tile_z = 80 with tile_y 32; tile_z = 160 with tile_y 24.  FP64: tile_z
 * = 32 with tile_y 8, 16 or 32; tile_z = 64 with tile_y 8, 16 or 24), the
 * number of x-planes per workgroup (chunk_x <= 0: library choice; the x
 * extent is split into equal chunks of at most chunk_x planes) and the column
 * group (col_group <= 0: library choice; that many column blocks of one patch
 * go to consecutive workgroups, so they share V_eff in the L2 cache) and the
 * column block (col_block: columns stepped by one workgroup, 1 or 2, sharing
 * the V_eff loads; 2 only on patches of at most 512 threads; 0: library
 * choice).  tile_z = tile_y = 0 restores the library's patch choice.  Applies
 * to blocks of every width.  The x split, the column group and the column
 * block never change results; another patch may change the last bits.  Not
 * thread-safe against calls that use the op.
 * Errors: SPARC_E_ARG (null op, bad dtype, unsupported tile, col_block
 * outside 0..2, or 2 on a patch of more than 512 threads). */
int sparc_op_set_launch(sparc_op *op, int32_t dtype, int32_t tile_z, int32_t tile_y, int32_t chunk_x,
                        int32_t col_group, int32_t col_block);

/* Measure the patch heights, a few x splits, column groups and column blocks
 * (1 or 2) of the vector step kernels for this op (its grid, atoms and projectors), dtype and
 * column count on scratch blocks (allocated and freed here), timing the launch
 * a filter step makes (projections in and out), apply the fastest to the op
 * for blocks of ns columns (other widths keep the library's choice), and
 * return it (out params may be NULL; best_us = microseconds per recurrence
 * step).  Results are cached per (grid, atoms, projectors, ns, dtype) in the
 * process and, when the environment variable SPARC_TUNE_CACHE names a file,
 * appended to and read from that file.  Synchronous.  Not thread-safe against
 * calls using the op.
 * Errors: SPARC_E_ARG, SPARC_E_SHAPE (the grid's z extent is not a multiple
 * of 4 FP32 / 2 FP64 nodes, or no patch plan is usable: nothing to tune),
 * SPARC_E_NOMEM, SPARC_E_HIP. */
int sparc_autotune(sparc_op *op, int32_t dtype, int32_t ns, void *stream, int32_t *tile_z, int32_t *tile_y,
                   int32_t *chunk_x, int32_t *col_group, int32_t *col_block, double *best_us);

/* Launch configuration of the step kernels for a dtype and ns as chosen by
 * the library for the op (out parameters may be NULL).  For grids the vector
 * kernels take: tile_z, tile_y, chunk_x, col_group and col_block of the
 * vector launch; otherwise the scalar kernels' patch (32 x 16), x-chunk and
 * col_group = col_block = 1. */
int sparc_step_config(const sparc_op *op, int32_t dtype, int32_t ns, int32_t *tile_z, int32_t *tile_y,
                      int32_t *chunk_x, int32_t *col_group, int32_t *col_block);

#ifdef __cplusplus
}
#endif
#endif /* SPARC_FILTER_H */
