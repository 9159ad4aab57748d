/*
 * dsw.h -- C-ABI of the MI355X direction-splitting library (libdsw.so).
 *
 * One time step of the direction-split nonlinear iteration of Frolov, Minev &
 * Takhirov, "An efficient algorithm for weakly compressible flows in spherical
 * geometries" (arXiv 2004.13887), section 2.2, eqs. (chapter3mainsd),
 * (splitting2) and (spl1)-(spl3), for the compressible Navier-Stokes system in
 * primitive variables U = [p, u_r, u_theta, u_phi, T] of section 2.1,
 * eqs. (nonconservmass)-(nonconservener) with the stiffened-gas equation of
 * state (nonconserveos), on a staggered (MAC) grid over a spherical shell
 * sector or the full sphere.  The direction operators D_r, D_theta, D_phi are
 * those of Appendix B, eqs. (dr), (dtheta), (dphi).
 *
 * Conventions
 * -----------
 * Every field argument is a dsw_fields of five DEVICE pointers (FP64), each a
 * dense C-order array (phi fastest):
 *     p, T : [n_r][n_theta][n_phi]           cell centres
 *     ur   : [n_r+1][n_theta][n_phi]         r faces
 *     ut   : [n_r][n_theta+1][n_phi]         theta faces
 *     uf   : [n_r][n_theta][n_phi_f]         phi faces, n_phi_f = n_phi if
 *                                            periodic_phi else n_phi + 1
 * Boundary-normal faces (r = r1, r2; theta walls or poles; phi walls) carry
 * Dirichlet velocities and are never changed by the library; they are 0 for
 * the no-slip walls and the poles this library implements.  Pressure and
 * temperature have zero normal gradient at every non-periodic boundary.  At a
 * pole (theta1 = 0 or theta2 = pi) u_theta = 0 on the pole face and the ghost
 * values are u_r: +interior, u_phi: -interior, p and T: +interior.
 *
 * The caller owns all field buffers (they must not alias unless stated) and
 * passes a HIP stream (hipStream_t as void*, NULL = the null stream); calls
 * enqueue work on that stream and return without synchronising.  A handle is
 * not thread safe; calls on one handle must be ordered (one stream).  The
 * library owns the handle, its metric tables and its workspace.
 *
 * Return codes: DSW_OK (0) or a negative DSW_E* code; dsw_last_error() gives
 * a thread-local message.  Device-side conditions (a vanishing pivot, a
 * non-positive temperature or p + pi_inf, a non-finite residual) set a
 * status word read by dsw_get_status().
 */
#ifndef DSW_H
#define DSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSW_OK 0
#define DSW_EINVAL (-1)    /* invalid argument or descriptor               */
#define DSW_ENOMEM (-2)    /* device allocation failed                     */
#define DSW_EHIP (-3)      /* a HIP runtime call failed                    */
#define DSW_ENONPHYS (-4)  /* finite T <= 0 or p + pi_inf <= 0 met         */
#define DSW_ESINGULAR (-5) /* zero pivot in a line solve                   */
#define DSW_EDIVERGED (-6) /* non-finite residual: the iteration diverged, or
                              the state holds a NaN or an infinity          */

/* Grid: n_r x n_theta x n_phi cells on [r1,r2] x [theta1,theta2] x [phi1,phi2]
 * (paper section 2.1, domain Omega).  Uniform spacing in r, theta and phi.
 * Requirements: all n >= 3; 0 < r1 < r2; 0 <= theta1 < theta2 <= pi;
 * phi1 < phi2; periodic_phi != 0 requires phi2 - phi1 = 2 pi (full sphere in
 * longitude; the phi line systems are then cyclic). */
typedef struct {
  int32_t n_r, n_theta, n_phi;
  int32_t periodic_phi;
  double r1, r2, theta1, theta2, phi1, phi2;
} dsw_grid_desc;

/* Material constants (paper section 2.1): c_p, c_v (gamma = c_p/c_v), the
 * stiffened-gas pi_inf, dynamic viscosity mu, Prandtl number, the rotation
 * rate omega about the polar axis, and the radial gravity g_r (the equations
 * carry +g on the left-hand side, so g_r > 0 pulls inward). */
typedef struct {
  double cp, cv, pi_inf, mu, prandtl, omega, g_r;
} dsw_material;

/* Five device pointers, layout as above. */
typedef struct {
  double *p, *ur, *ut, *uf, *T;
} dsw_fields;

/* Element counts and shapes of the five arrays (order p, ur, ut, uf, T). */
typedef struct {
  int64_t shape[5][3];
  int64_t count[5];
  int64_t bytes_per_state; /* sum of the five arrays in bytes */
} dsw_layout_info;

typedef struct dsw_grid dsw_grid;

/* Validate the descriptors, build the metric tables and allocate the
 * workspace on the current HIP device.  *out receives the handle.
 * Errors: DSW_EINVAL, DSW_ENOMEM, DSW_EHIP. */
int dsw_init_grid(const dsw_grid_desc *desc, const dsw_material *mat, dsw_grid **out);

/* Release the handle and its device memory (synchronises the device). */
int dsw_free_grid(dsw_grid *grid);

/* Shapes and sizes of the field arrays the caller must allocate. */
int dsw_layout(const dsw_grid *grid, dsw_layout_info *info);

/* Right-hand side of eq. (spl1), simplified: with Ubar = (Uk + Un)/2,
 *   R = -(Uk - Un) - tau * F_h(Ubar),  F_h(V) = (D + D_M)(V) V + G
 * (D, D_M, G of eq. (chapter3main)), at every unknown; R = 0 on
 * boundary-normal faces.  Ubar is written everywhere.  Un, Uk: inputs
 * (may alias each other); R, Ubar: outputs (must not alias the inputs). */
int dsw_residual(dsw_grid *grid, const dsw_fields *Un, const dsw_fields *Uk, double tau,
                 dsw_fields *R, dsw_fields *Ubar, void *stream);

/* Line solves of eqs. (spl1), (spl2), (spl3): x = (I + tau/2 D_d(Ubar))^{-1} rhs
 * for d = r, theta, phi, with homogeneous increment boundary conditions.  Each
 * line carries one 3x3-block tridiagonal system in (p, T, u_d) and one scalar
 * tridiagonal system per transverse velocity; _phi is cyclic when the grid is
 * periodic.  rhs must be 0 on boundary-normal faces; x is 0 there.
 * rhs and x must not alias. */
int dsw_line_solve_r(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                     dsw_fields *x, void *stream);
int dsw_line_solve_theta(dsw_grid *grid, const dsw_fields *Ubar, double tau,
                         const dsw_fields *rhs, dsw_fields *x, void *stream);
int dsw_line_solve_phi(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                       dsw_fields *x, void *stream);

/* One split time step (eqs. (spl1)-(spl3) iterated K times, U^{n+1,0} = U^n,
 * U^{n+1} = U^{n+1,K}): Unp1 receives U^{n+1}.  Un is not modified; Unp1 must
 * not alias Un.  K >= 1, tau > 0.  Uses the handle's workspace. */
int dsw_split_step(dsw_grid *grid, const dsw_fields *Un, dsw_fields *Unp1, double tau, int32_t K,
                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as dsw_split_step, with the same results, that allocates nothing.  Its
 * workspace (two midpoint states, the residual, the outputs of the r and
 * theta sweeps, the sweep scratch) lives in one library-owned device array of
 * DSW_NOALLOC_BYTES per GPU, which each GPU the library runs on holds until
 * the process ends (its address is taken at dsw_init_grid).  A grid whose
 * workspace exceeds it (about 5 x 8 x (cells + faces) + 8 x 27 x cells bytes;
 * some 640 thousand cells fit) is refused with DSW_EINVAL and nothing is
 * enqueued.  The handle's device must be current, else DSW_EINVAL.  All calls
 * on one GPU share the array: calls that overlap in time on one GPU (two
 * streams, two threads, two handles) race and give undefined results; calls
 * ordered on one stream are safe.  Every part of the array a call reads it
 * has first written, so no clearing is needed between calls. */
#define DSW_NOALLOC_BYTES (256LL * 1024 * 1024)
int dsw_split_step_noalloc(dsw_grid *grid, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                           int32_t K, void *stream);

/* Tangential velocities on the non-periodic walls at one time level.  Device
 * arrays, C order; a null entry is a zero wall velocity.  A ghost value
 * across a wall is 2 g - u of the interior neighbour (the no-slip rule of the
 * velocity boundary condition, paper section 2.1, with the wall moving).  Pole
 * boundaries ignore them (symmetry ghosts).
 *   ur_t1, ur_t2 [n_r+1][n_phi]      u_r on the theta = theta1 / theta2 walls
 *   ur_p1, ur_p2 [n_r+1][n_theta]    u_r on the phi = phi1 / phi2 walls
 *   ut_r1, ut_r2 [n_theta+1][n_phi]  u_theta on the r = r1 / r2 walls
 *   ut_p1, ut_p2 [n_r][n_theta+1]    u_theta on the phi walls
 *   uf_r1, uf_r2 [n_theta][npf]      u_phi on the r walls
 *   uf_t1, uf_t2 [n_r][npf]          u_phi on the theta walls
 * (npf = n_phi + 1 on a sector, n_phi when periodic). */
typedef struct {
  const double *ur_t1, *ur_t2, *ur_p1, *ur_p2;
  const double *ut_r1, *ut_r2, *ut_p1, *ut_p2;
  const double *uf_r1, *uf_r2, *uf_t1, *uf_t2;
} dsw_wall;

/* dsw_split_step with forcing and time-dependent velocity boundary data, for
 * manufactured solutions (paper section 3.1, eq. (man_sol)) and moving walls:
 *   src   (may be NULL, as may each of its arrays) a source S added to the
 *         right-hand side of the system, taken at the midpoint time: every
 *         iteration's residual is -(U^k - U^n) - tau (F_h(Ubar) - S);
 *   wall0, wall1 (each may be NULL) tangential wall velocities at t^n and
 *         t^{n+1};
 *   bnd   (may be NULL) fields whose boundary-normal faces (ur, ut, uf; p and
 *         T are not read) hold the Dirichlet data of t^{n+1}; Un's hold those
 *         of t^n.  NULL: the data keep Un's.
 * U^{n+1,0} = U^n, boundary data included (eq. (chapter3mainsd)).  The first
 * iteration's increment solves (spl1)-(spl3) carry the change of the boundary
 * data to t^{n+1} as inhomogeneous Dirichlet data of the increments (lifted
 * into their right-hand sides); every later iterate holds the new data, its
 * midpoint their mean with Un's, and its ghost values the mean wall velocity.
 * The rest as dsw_split_step.  Runs the residual over every point and needs
 * phi lines that the partitioned solver takes (any sector of up to 1024 phi
 * cells; on a full sphere a power-of-two chunk count), else DSW_EINVAL.  The
 * first call on a handle allocates a small workspace for the wall data. */
int dsw_split_step_forced(dsw_grid *grid, const dsw_fields *Un, dsw_fields *Unp1, double tau,
                          int32_t K, const dsw_fields *src, const dsw_wall *wall0,
                          const dsw_wall *wall1, const dsw_fields *bnd, void *stream);

/* Perturbation-pressure form (paper section 3.1, the remark after Table 3:
 * with a large background pressure the errors of the pressure derivatives
 * scale with it, and the pressure is rescaled a priori).  The state's p
 * array holds p' = p - p_ref(r) instead of p, for a reference column
 * (p_ref_i, T_ref_i) at the cell centres that is discretely hydrostatic under
 * the radial momentum row at rest:
 *   (p_ref_i - p_ref_{i-1}) / dr + g_r (rho_ref_{i-1} + rho_ref_i) / 2 = 0,
 *   rho_ref_i = (p_ref_i + pi_inf) / ((c_p - c_v) T_ref_i).
 * dsw_split_step_pert computes the step of dsw_split_step with that balance
 * subtracted analytically: coefficients see p' + p_ref; the radial row's
 * pressure gradient plus gravity is the gradient of p' plus the buoyancy
 * g_r (rho_f - rho_ref_f) / rho_f, formed without a difference of large
 * numbers; the advection of p gains u_r d p_ref / dr.  In exact arithmetic
 * it equals dsw_split_step on p = p' + p_ref; in FP64 the pressure change
 * keeps its relative precision at any background pressure, and a fluid at
 * rest in an isothermal reference column stays exactly at rest.
 *   dsw_set_reference  p_ref, T_ref: host arrays of n_r doubles (copied; the
 *                      caller keeps them).  The discrete balance above is the
 *                      caller's to satisfy: the step subtracts it as if
 *                      exact.  DSW_EINVAL if p_ref + pi_inf or T_ref is not
 *                      positive and finite; DSW_ENOMEM.
 *   dsw_split_step_pert  Un, Unp1 as for dsw_split_step, p fields in the
 *                      perturbation form; DSW_EINVAL before a reference is
 *                      set.  Plain walls (no forcing); timed like
 *                      dsw_split_step when timing is enabled. */
int dsw_set_reference(dsw_grid *grid, const double *p_ref, const double *T_ref);
int dsw_split_step_pert(dsw_grid *grid, const dsw_fields *Un, dsw_fields *Unp1, double tau, int32_t K,
                        void *stream);

/* Courant numbers of a state for a step tau, for a time-step controller
 * (paper section 3.2: once the Thermal 1 bubble accelerates, the step must
 * shrink or adapt).  At every cell centre, with the centre-averaged
 * velocity and the spacings h_r = dr, h_t = r dtheta, h_f = r sin(theta) dphi:
 *   out[0] = max tau (|u_r| / h_r + |u_theta| / h_t + |u_phi| / h_f)  (advective)
 *   out[1] = max tau c max(1/h_r, 1/h_t, 1/h_f), c = sqrt(gamma R T) (acoustic).
 * U: device state (the p field is not read, so either pressure form works);
 * out: host, 2 doubles.  Synchronises the stream.  The first call allocates
 * 16 bytes of device memory kept with the grid.  DSW_EINVAL for null
 * arguments or tau <= 0. */
int dsw_courant(dsw_grid *grid, const dsw_fields *U, double tau, double out[2], void *stream);

/* Optional per-kernel timing of dsw_split_step.  While enabled, every kernel
 * the step enqueues is bracketed by a pair of HIP events recorded on the same
 * stream.  dsw_read_timing synchronises that stream, stores in ms[kind] the
 * total elapsed time and in launches[kind] the number of launches recorded
 * since the previous read (kind 0: residual, 1: r sweep, 2: theta sweep,
 * 3: phi sweep with update, 4: copy of the Dirichlet boundary faces), then
 * clears the record.  If an elapsed time cannot be read (e.g. the step ran on
 * another stream that is still busy), it returns DSW_EHIP and keeps the
 * record and its events for a later read. */
#define DSW_TIMING_KINDS 5
int dsw_set_timing(dsw_grid *grid, int32_t enable);
int dsw_read_timing(dsw_grid *grid, void *stream, double ms[DSW_TIMING_KINDS],
                    int64_t launches[DSW_TIMING_KINDS]);

/* Adjoint (reverse mode) of dsw_split_step.  The split step is a map
 * Phi: U^n -> U^{n+1} (paper eqs. (spl1)-(spl3), K iterations); its Jacobian
 * J is taken exactly as the discrete map is written, every iteration's
 * midpoint linearisation and line matrices included (a discrete, not a
 * continuous, adjoint).
 *
 * dsw_adjoint_step: lam_n = J(U^n)^T lam_np1 over every array entry (the
 *   boundary-normal faces included: their entries of U^{n+1} are copies of
 *   those of U^n).  Un is the checkpoint of the step; the forward step is
 *   recomputed from it, keeping each iteration's midpoint and line-solve
 *   outputs in a workspace of 4K+7 states and a second sweep scratch that
 *   the handle allocates on the first call (and grows for a larger K).  The
 *   last iteration's transposed solves run on a second stream of the handle
 *   (non-blocking, default priority) beside the recompute's last iteration;
 *   the call orders that work before its later work on `stream`, so the
 *   caller sees one stream.  lam_n must not alias Un or lam_np1.  tau, K:
 *   those of the forward step.
 *
 * The pieces, exported for tests and for custom reverse passes:
 * dsw_line_solve_T_{r,theta,phi}: x = (I + tau/2 D_d(Ubar))^{-T} rhs, the
 *   transposed line systems (block, scalar; cyclic on a periodic grid), same
 *   conventions as dsw_line_solve_*.
 * dsw_line_vjp_{r,theta,phi}: acc += (d[(I + tau/2 D_d(Ubar)) X]/dUbar)^T mu,
 *   the transposed derivative of the line operator applied to a fixed X,
 *   with respect to the state it is linearised at.
 * dsw_residual_vjp: acc += (d[-tau F_h(Ubar)]/dUbar)^T mu, mu taken at the
 *   unknowns (the rows of the boundary-normal faces are constant).
 * The _vjp calls accumulate with FP64 atomic adds: acc must be initialised
 * by the caller, and the last bits of the sums may vary from run to run. */
int dsw_adjoint_step(dsw_grid *grid, const dsw_fields *Un, double tau, int32_t K,
                     const dsw_fields *lam_np1, dsw_fields *lam_n, void *stream);
int dsw_line_solve_T_r(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                       dsw_fields *x, void *stream);
int dsw_line_solve_T_theta(dsw_grid *grid, const dsw_fields *Ubar, double tau,
                           const dsw_fields *rhs, dsw_fields *x, void *stream);
int dsw_line_solve_T_phi(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *rhs,
                         dsw_fields *x, void *stream);
int dsw_line_vjp_r(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                   const dsw_fields *mu, dsw_fields *acc, void *stream);
int dsw_line_vjp_theta(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                       const dsw_fields *mu, dsw_fields *acc, void *stream);
int dsw_line_vjp_phi(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *X,
                     const dsw_fields *mu, dsw_fields *acc, void *stream);
int dsw_residual_vjp(dsw_grid *grid, const dsw_fields *Ubar, double tau, const dsw_fields *mu,
                     dsw_fields *acc, void *stream);

/* The adjoint step without the forward recompute, for callers that keep a
 * tape of the forward step (e.g. a backward pass right after the forward
 * one).  The tape holds what the reverse of every iteration reads: the
 * midpoint and the outputs X1, X2, X3 of the three line solves (4K
 * five-field states; caller-owned device memory of dsw_tape_bytes bytes,
 * 8-byte aligned, one tape per recorded step).
 * dsw_tape_bytes: the size of the tape of a K-iteration step.
 * dsw_split_step_taped: dsw_split_step (the same kernels and result) that
 *   also fills the tape.
 * dsw_adjoint_step_taped: dsw_adjoint_step from a tape filled by
 *   dsw_split_step_taped with the same Un, tau and K (the tape is read only;
 *   the result is that of dsw_adjoint_step up to the order of the atomic
 *   sums). */
int dsw_tape_bytes(const dsw_grid *grid, int32_t K, int64_t *bytes);
int dsw_split_step_taped(dsw_grid *grid, const dsw_fields *Un, dsw_fields *Unp1, double tau, int32_t K,
                         void *tape, void *stream);
int dsw_adjoint_step_taped(dsw_grid *grid, const dsw_fields *Un, double tau, int32_t K,
                           const void *tape, const dsw_fields *lam_np1, dsw_fields *lam_n, void *stream);

/* The adjoint of nsteps consecutive split steps (a trajectory U^0 -> U^N,
 * N = nsteps, with a checkpoint of every step's starting state): lam_0 =
 * J(U^0)^T ... J(U^{N-1})^T lam_end, i.e. dsw_adjoint_step applied from the
 * last step back to the first, each step recomputed from its checkpoint.
 * ckpts: host array of N field descriptors, ckpts[n] = U^n on the device
 * (read only).  lam_end: the cotangent of U^N; lam_0: the result, which
 * must alias neither lam_end nor a checkpoint.  The recompute of step n-1
 * runs on a second stream of the handle while the reverse of step n runs on
 * `stream` (the two read and write disjoint buffers); every piece of work is
 * ordered before the call's later work on `stream`.  Workspace: 8K+9 states
 * and a second sweep scratch, allocated by the handle on first use.  The
 * result equals N chained dsw_adjoint_step calls up to the order of the
 * atomic sums.  Errors: those of dsw_adjoint_step; DSW_EINVAL for
 * nsteps < 1 or a null ckpts. */
int dsw_adjoint_trajectory(dsw_grid *grid, const dsw_fields *ckpts, int32_t nsteps, double tau, int32_t K,
                           const dsw_fields *lam_end, dsw_fields *lam_0, void *stream);

/* Launch shapes of a grid's kernels (the tunable parameters; they change
 * speed and the order of rounding, never the method):
 *   residual_block        threads per workgroup of the residual (64, 128, 256)
 *   sweep_block_r/_theta  threads per workgroup of the r / theta sweeps
 *                         (64, 128, 256)
 *   phi_rows_per_thread   phi sweep: 2 or 4 = partitioned solver, one
 *                         workgroup per line, that many rows per thread,
 *                         separators by cyclic reduction in LDS; 0 = one
 *                         thread per line.  Lines the partitioned solver
 *                         cannot take (more than 256 chunks, or a cyclic line
 *                         whose chunk count is not a power of two) fall back
 *                         to one thread per line.  The transposed phi
 *                         solves of the adjoint take two rows per thread
 *                         wherever the line allows it.
 *   rows_per_thread_r/_theta
 *                         r / theta sweeps: 4 = partitioned solver (each
 *                         workgroup on a few neighbouring lines split into
 *                         chunks, 4 rows per thread on the 3x3-block lines
 *                         and 8 on the scalar ones, separators by cyclic
 *                         reduction in LDS; no scratch memory); 0 = two
 *                         threads per line, eliminating from both ends,
 *                         intermediates in a scratch array (the scalar
 *                         lines of lines with 64, 128 or 256 rows run
 *                         apart, by the partitioned solver); -1 = by line
 *                         length: partitioned where a line has at most 128
 *                         rows (32 chunks), else two-ended (in an ensemble,
 *                         member by member).  Lines of more than
 *                         4 x sweep_block rows take the two-ended solver.
 *                         The transposed r solves of the adjoint take the
 *                         same solver; the transposed theta solves always
 *                         the two-ended one.  Measured: partitioned r
 *                         0.16 ms, theta 0.19 ms against 0.20 / 0.31 ms
 *                         two-ended on the 256 x 128 x 64 sector; on the
 *                         512 x 256 x 128 sphere r 1.37 / 1.37 ms (2.4x
 *                         fewer HBM bytes partitioned) and theta 1.71 /
 *                         1.43 ms.
 * Default {64, 256, 256, 4, -1, -1}.  dsw_set_config returns DSW_EINVAL for
 * other values.  dsw_ensemble_tune times candidate shapes per pass and keeps
 * each pass's best; its result is also kept for the process per set of member
 * shapes and K, and a later tuning of the same shapes returns it untimed. */
typedef struct {
  int32_t residual_block, sweep_block_r, sweep_block_theta, phi_rows_per_thread;
  int32_t rows_per_thread_r, rows_per_thread_theta;
} dsw_config;
int dsw_set_config(dsw_grid *grid, const dsw_config *cfg);
int dsw_get_config(const dsw_grid *grid, dsw_config *cfg);

/* Ensembles: n independent grids (uneven sizes allowed) stepped together.
 * Each member is a full grid handle with its own workspace; a step of the
 * ensemble computes exactly what dsw_split_step computes for every member
 * (paper section 2.2, eqs. (spl1)-(spl3) iterated K times), with one launch
 * per pass covering all members of a lane (workgroups mapped to members by
 * a table of offsets) instead of one launch per member and pass, and the
 * whole step captured once in a HIP graph and replayed.  The graph holds two
 * lanes of members (balanced by cells) as two chains of launches, the
 * second starting after the first lane's first residual launch, so that
 * their passes overlap; the graph runs on the caller's stream as one unit.
 *
 * dsw_ensemble_create: descs and mats are arrays of n (n >= 1).
 * dsw_ensemble_member: borrowed handle of member m (valid until the ensemble
 *   is freed; do not free it); use it for dsw_layout or single-grid calls.
 * dsw_ensemble_step: Un, Unp1 and tau are arrays of n; member m steps
 *   Un[m] -> Unp1[m] with tau[m] (same rules as dsw_split_step).  The first
 *   call with a given set of pointers, steps and K builds and captures the
 *   graph (a few ms); later calls replay it.  At most 8 such graphs are
 *   kept (the oldest is dropped, after a device synchronisation).
 * dsw_ensemble_tune: an autotuner.  It runs the batched step directly (no
 *   graph) under candidate launch shapes, `reps` timed steps each, times every
 *   pass with HIP events, and keeps for each pass the fastest shape.  The
 *   result becomes the configuration of the ensemble and of every member
 *   (so that per-member dsw_split_step calls compute the same numbers) and
 *   is stored in *best if best is non-NULL.  Unp1 is overwritten.
 *   Synchronises the stream.  Candidates: each workgroup width with its
 *   phi solver, and the r / theta solvers all partitioned, all two-ended or
 *   by line length member by member.  The result is kept for the process per
 *   set of member shapes and K; tuning the same shapes again returns it
 *   without running anything.
 * dsw_ensemble_get_status: dsw_get_status over all members (first error). */
typedef struct dsw_ensemble dsw_ensemble;
int dsw_ensemble_create(const dsw_grid_desc *descs, const dsw_material *mats, int32_t n,
                        dsw_ensemble **out);
int dsw_ensemble_free(dsw_ensemble *ens);
int dsw_ensemble_member(dsw_ensemble *ens, int32_t m, dsw_grid **grid);
int dsw_ensemble_step(dsw_ensemble *ens, const dsw_fields *Un, dsw_fields *Unp1, const double *tau,
                      int32_t K, void *stream);
int dsw_ensemble_tune(dsw_ensemble *ens, const dsw_fields *Un, dsw_fields *Unp1, const double *tau,
                      int32_t K, int32_t reps, void *stream, dsw_config *best);
int dsw_ensemble_set_config(dsw_ensemble *ens, const dsw_config *cfg);
int dsw_ensemble_get_config(const dsw_ensemble *ens, dsw_config *cfg);
int dsw_ensemble_get_status(dsw_ensemble *ens, void *stream);

/* Synchronise the stream, read and clear the device status word.  Returns
 * DSW_OK, or the first of DSW_ENONPHYS, DSW_EDIVERGED, DSW_ESINGULAR that
 * was met (or DSW_EHIP).  A non-finite residual ranks before a singular
 * pivot: the line solves that follow it meet non-finite pivots too. */
int dsw_get_status(dsw_grid *grid, void *stream);

/* Thread-local description of the last error (never NULL). */
const char *dsw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DSW_H */
