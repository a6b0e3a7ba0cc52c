/*
 * rsfde.h — C ABI of the MI355X (gfx950) solver for the volume-penalized
 * implicit finite-difference system of the 2-D Riesz space-fractional
 * diffusion equation, preconditioned by the sine-transform (tau) matrices
 * (and its 3-D form, rsfde_setup3).
 *
 * Paper: X. Huang, H.-W. Sun, "A preconditioner based on sine transform for
 * two-dimensional Riesz space fractional diffusion equations in convex
 * domains", arXiv 2102.11576.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: n1 x n2 interior points of the box (x_lo,x_hi) x (y_lo,y_hi),
 *    h_x = (x_hi-x_lo)/(n1+1), h_y = (y_hi-y_lo)/(n2+1)  (Section 2).
 *  - Vectors are FP64 device arrays of N = n1*n2 entries in row-major
 *    [n2][n1] order (x fastest) — the lexicographic ordering of Section 2.
 *    They are owned by the caller, must not overlap unless stated, and must
 *    stay valid until the call returns.
 *  - mask: uint8 device array [n2][n1], 1 = grid point inside the convex
 *    domain, 0 = penalty region (the paper's Phi_d is diag(1 - mask)).
 *  - stream: a hipStream_t passed as void* (NULL = the stream given at setup).
 *    All device work of a call is enqueued on that stream.  Calls that run the
 *    Krylov solver return after the solve has finished (the host takes the
 *    convergence decisions); matvec / precond_apply return after enqueueing.
 *  - Every function returns RSFDE_OK (0) or a negative error code; no C++
 *    exception crosses the ABI.  Arguments are validated on the host before
 *    any device work is enqueued.
 *  - A plan is bound to the device that was current at setup, holds all of
 *    its workspaces (no allocation after setup), and is not thread-safe.
 */
#ifndef RSFDE_H
#define RSFDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define RSFDE_OK 0
#define RSFDE_EINVAL (-1)       /* invalid argument (checked before any device work) */
#define RSFDE_ENOMEM (-2)       /* device or pinned-host allocation failed at setup */
#define RSFDE_EHIP (-3)         /* a HIP runtime call failed */
#define RSFDE_ENOTCONV (-4)     /* iteration cap reached; output holds the last iterate */
#define RSFDE_EBREAKDOWN (-5)   /* Arnoldi breakdown with the true residual above tol */
#define RSFDE_ENONFINITE (-6)   /* NaN or Inf in the input or in the Krylov recurrence */
#define RSFDE_EUNSUPPORTED (-7) /* valid but not implemented for this shape / option */

/* precision of the preconditioner apply (the rest of the solve is FP64) */
#define RSFDE_FP64 0
#define RSFDE_FP32 1
#define RSFDE_BF16 2

/* preconditioner */
#define RSFDE_PRECOND_TAU 0  /* the sine-transform preconditioner P_hat (Section 4.1) */
#define RSFDE_PRECOND_NONE 1 /* plain GMRES */

/* nonlinear source term f(u) (zero outside the domain, Section 2) */
#define RSFDE_F_NONE 0     /* f = 0 */
#define RSFDE_F_LOGISTIC 1 /* f = u (1 - u) */
#define RSFDE_F_SIN 2      /* f = sin u */
#define RSFDE_F_CUBIC 3    /* f = u - u^3 */
#define RSFDE_F_DECAY 4    /* f = -u (with a source field: Example 1 of Section 5) */

/* preconditioning side (rsfde_solver_opts.side) */
#define RSFDE_ZSTORE_FP64 0
#define RSFDE_ZSTORE_FP32 1
#define RSFDE_RIGHT 0 /* flexible GMRES on M P^{-1}; stop on ||b - M x|| <= tol ||b|| */
#define RSFDE_LEFT 1  /* GMRES on P^{-1} M; stop on the estimate of ||P^{-1}(b - M x)||
                         <= tol ||P^{-1} b||: the stopping rule of Section 5 */

typedef struct rsfde_plan_s* rsfde_plan;

typedef struct {
  int32_t n1, n2;           /* interior points in x and y, >= 1 */
  double x_lo, x_hi;        /* box in x, x_hi > x_lo */
  double y_lo, y_hi;        /* box in y, y_hi > y_lo */
} rsfde_grid;

typedef struct {
  int32_t restart;   /* GMRES restart length, 1 .. max_restart of the plan */
  int32_t max_iters; /* cap on inner iterations per solve (>= 1) */
  double tol;        /* relative tolerance > 0 of the stopping rule of `side` */
  int32_t precision; /* RSFDE_FP64 / RSFDE_FP32 / RSFDE_BF16: preconditioner arithmetic */
  int32_t precond;   /* RSFDE_PRECOND_TAU or RSFDE_PRECOND_NONE */
  int32_t reorth;    /* Gram-Schmidt passes of the one-vector form: 0 (default) or
                        1 = two (CGS2), -1 = one (CGS) */
  int32_t side;      /* RSFDE_RIGHT (default) or RSFDE_LEFT; with RSFDE_PRECOND_NONE
                        both are plain GMRES */
  int32_t sstep;     /* 0 or 1: one Arnoldi vector per step (classical Gram-Schmidt).
                        2..16: s-step form (right side, sine-transform preconditioner):
                        s directions u_{i+1} = (M P^{-1} - I) u_i per block, orthogonalised
                        together (block Gram-Schmidt + Cholesky QR); same Krylov space,
                        about s times less basis traffic.  Grids with N < 4096 use the
                        one-vector form. */
  int32_t zstore;    /* storage of the preconditioned basis Z of the flexible GMRES:
                        RSFDE_ZSTORE_FP64 (default) or RSFDE_ZSTORE_FP32.  With FP32
                        each z_j is rounded when stored and w_j = M z_j is formed from
                        the stored vector, so the Arnoldi relation M Z = V H holds for
                        the kept basis and the true-residual stop is unchanged; the
                        basis reads of the solution update and the product's z reads
                        halve.  Right side, sine-transform preconditioner (FP64 or
                        FP32), two-dimensional plans with n1+1 and n2+1 powers of two
                        (EUNSUPPORTED otherwise). */
} rsfde_solver_opts;

typedef struct {
  int32_t iters;      /* inner (Arnoldi) iterations used by the solve */
  int32_t restarts;   /* restart cycles started */
  int32_t status;     /* same code as the return value */
  int32_t reserved;
  double relres;      /* relative residual at exit: true ||b - M x|| / ||b|| (right), or
                         the estimate of ||P^{-1}(b - M x)|| / ||P^{-1} b|| (left) */
  double bnorm;       /* ||b||_2 (right) or ||P^{-1} b||_2 (left) */
} rsfde_stats;

/*
 * Create a plan: GL weights (g_form), c_alpha = -1/(2 cos(alpha pi/2)),
 * c_x = dt kx c_alpha1 / h_x^alpha1 and c_y likewise (Section 2), the Toeplitz
 * first columns of (G), the circulant-embedding symbols used by the O(N log N)
 * matrix-vector product, and the tau-matrix eigenvalues diagonalised by the
 * sine transform (Section 4.1).  Copies the mask (N bytes) into plan memory.
 *   out         : receives the plan (set to NULL on error)
 *   grid        : host pointer
 *   alpha1/2    : fractional orders, 1 < alpha < 2
 *   kx, ky      : diffusion coefficients, >= 0 (can be changed later)
 *   mask_dev    : device pointer [n2][n1]
 *   eta, dt     : penalty parameter > 0 and time step > 0
 *   max_restart : largest restart the plan will run (1..64; <= 0 means 30)
 *   stream      : stream for the set-up uploads
 * Any n1, n2 from 1 to 4096 (EUNSUPPORTED above).  When n1+1 and n2+1 are
 * powers of two the FP64 / FP32 preconditioner runs its sine transforms as
 * FFTs of the odd extension (length 2(n+1)); otherwise as chirp convolutions
 * (Bluestein) on power-of-two FFTs of length >= 2n-1, about four times the
 * arithmetic for the same result.
 * Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED.
 */
int rsfde_setup(rsfde_plan* out, const rsfde_grid* grid, double alpha1, double alpha2,
                double kx, double ky, const uint8_t* mask_dev, double eta, double dt,
                int32_t max_restart, void* stream);

/* Three-dimensional plans.  The paper treats two dimensions and leaves higher
 * dimensions to future work (concluding section); this plan carries Section 2
 * and Section 4.1 over with a third Kronecker factor:
 *   M = I - (I (x) I (x) A_x + I (x) A_y (x) I + A_z (x) I (x) I) + D,
 *   P_hat^{-1} = mask (S (x) S (x) S)(I - Lx - Ly - Lz)^{-1}(S (x) S (x) S)
 *              + (1 - mask) (S (x) S (x) S)((1 + dt/eta) I - Lx - Ly - Lz)^{-1}(S (x) S (x) S)
 * with A_z = c_z G^(alpha3), c_z = dt kz c_alpha3 / h_z^alpha3, and the tau
 * eigenvalues along each axis.  Vectors and the mask are [n3][n2][n1] (x
 * fastest), N = n1 n2 n3.  Each n <= 4095 (EUNSUPPORTED otherwise) and
 * (n1+1) n2 n3 < 2^31.  When n1+1, n2+1 and n3+1 are all powers of two the
 * sine transforms are odd-extension FFTs; otherwise every axis takes the chirp
 * (Bluestein) form of the DST-I, as rsfde_setup does for other n.
 * rsfde_matvec, rsfde_precond_apply (FP64 / FP32), rsfde_step, rsfde_step_src,
 * rsfde_solve, rsfde_march_ensemble, rsfde_set_coeffs / rsfde_set_coeffs3 and
 * rsfde_adjoint_step (three k gradients) accept a 3-D plan; the BF16
 * preconditioner returns EUNSUPPORTED for it.
 * The plan owns four preconditioner intermediates of (n1+1) n2 n3 doubles and
 * one more vector than a 2-D plan.  Other arguments as rsfde_setup.
 * Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED. */
typedef struct {
  int32_t n1, n2, n3;       /* interior points in x, y, z, >= 1 */
  double x_lo, x_hi;
  double y_lo, y_hi;
  double z_lo, z_hi;        /* box in z, z_hi > z_lo */
} rsfde_grid3;

int rsfde_setup3(rsfde_plan* out, const rsfde_grid3* grid, double alpha1, double alpha2,
                 double alpha3, double kx, double ky, double kz, const uint8_t* mask_dev,
                 double eta, double dt, int32_t max_restart, void* stream);

/* Change kx, ky (Section 2's diffusion coefficients, constant here).  2-D
 * plans: O(1), the symbols and eigenvalues are stored for k = 1 and scaled at
 * apply time.  3-D plans: kz is kept; see rsfde_set_coeffs3.
 * Errors: EINVAL (negative or non-finite k), EHIP. */
int rsfde_set_coeffs(rsfde_plan plan, double kx, double ky);

/* Change kx, ky, kz of a 3-D plan.  kz is applied at launch; the
 * preconditioner's folded x/y eigenvalue table carries kx and ky, so when they
 * change it is rebuilt on the host and copied in after hipDeviceSynchronize
 * (the call blocks; no work of the plan may be enqueued from another thread
 * meanwhile).  A 2-D plan accepts kz = 0 only (as rsfde_set_coeffs).
 * Errors: EINVAL (negative or non-finite k, kz != 0 on a 2-D plan), EHIP (the
 * plan then keeps its previous kx, ky). */
int rsfde_set_coeffs3(rsfde_plan plan, double kx, double ky, double kz);

/* y = M x with M = I - A + D, A = I (x) A_x + A_y (x) I (matrix_vector,
 * toeplitz_A): two FFT-convolution passes.  x and y must not overlap.
 * Errors: EINVAL, EHIP. */
int rsfde_matvec(rsfde_plan plan, const double* x, double* y, void* stream);

/* y = M x as rsfde_matvec, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): no plan, and no allocation of any kind.  The grid, orders,
 * coefficients, mask (device, [n2][n1], 1 = in Omega), eta and dt are those of
 * rsfde_setup; x, y are device [n2][n1] FP64 arrays owned by the caller and
 * must not overlap.  Work is enqueued on `stream` (NULL: the null stream) on
 * the current device.
 * Scratch: one library-owned device array of 33 MiB per device (loaded with
 * the code object, held until the process ends) holds the row-pass
 * intermediate and the symbol and twiddle tables.  Limit: n1, n2 <= 2047.
 * The symbol and twiddle tables are rebuilt on the device (one more kernel on
 * `stream`, no host transfer) only when the grid, alpha1/alpha2 or the unit
 * coefficients dt c_alpha / h^alpha change from the previous call on the
 * device; otherwise the call enqueues the two kernels of the product.  The
 * call never blocks the host.  Every call on a device shares that array:
 * calls that overlap on one device (other streams, other host threads) race.
 * Results equal rsfde_matvec's to rounding (the tables are the same sums,
 * evaluated on the device).
 * Errors: EINVAL (bad argument), EUNSUPPORTED (grid beyond the limit), EHIP. */
int rsfde_matvec_noalloc(const rsfde_grid* grid, double alpha1, double alpha2, double kx,
                         double ky, const uint8_t* mask_dev, double eta, double dt,
                         const double* x, double* y, void* stream);

/* z = P_hat^{-1} r (preconditioner): 2-D DST-I, the two eigenvalue scalings
 * 1/(1 - lx_i - ly_j) and 1/(1 + dt/eta - lx_i - ly_j), inverse 2-D DST-I,
 * combined by the mask.  precision selects the internal arithmetic: FP64 or
 * FP32 run the transforms as FFTs (odd extension when n+1 is a power of two,
 * chirp convolution otherwise); BF16 runs them as dense sine-matrix products
 * on the matrix cores (BF16 operands, FP32 accumulation).  Any n.  r and z
 * must not overlap.
 * Errors: EINVAL, EHIP. */
int rsfde_precond_apply(rsfde_plan plan, const double* r, double* z, int32_t precision,
                        void* stream);

/* One implicit time step (difference_scheme / linearsystem):
 *   b = u_prev + dt * mask * f(u_prev),  solve M u_next = b
 * by restarted GMRES (opts->side: right-preconditioned flexible GMRES, or the
 * left-preconditioned form of Section 5), initial guess 2 u_prev - u_prev2
 * (u_prev if u_prev2 is NULL) as in Section 5.
 * u_next may alias u_prev2 (but not u_prev).  stats may be NULL.
 * Errors: EINVAL, ENOTCONV (u_next holds the last iterate), ENONFINITE, EHIP. */
int rsfde_step(rsfde_plan plan, const double* u_prev, const double* u_prev2, int32_t f_kind,
               const rsfde_solver_opts* opts, double* u_next, rsfde_stats* stats,
               void* stream);

/* rsfde_step with an x,y,t-dependent source field (Section 2 allows f to depend
 * on x, y and t; Example 1 of Section 5 is f = -u + g(x, y, t)):
 *   b = u_prev + dt * mask * (f(u_prev) + src_scale * src)
 * src: device array [n2][n1] (NULL: no field term, as rsfde_step), read only;
 * src_scale: finite scalar (e.g. a time factor, so one stored field serves
 * every step of a separable source).  src must not alias u_next.
 * Errors: as rsfde_step. */
int rsfde_step_src(rsfde_plan plan, const double* u_prev, const double* u_prev2, int32_t f_kind,
                   const double* src, double src_scale, const rsfde_solver_opts* opts,
                   double* u_next, rsfde_stats* stats, void* stream);

/* Solve M x = b for a caller-supplied right-hand side (used by the adjoint
 * and by tests).  x holds the initial guess on entry and the solution on exit.
 * Errors: as rsfde_step. */
int rsfde_solve(rsfde_plan plan, const double* b, double* x, const rsfde_solver_opts* opts,
                rsfde_stats* stats, void* stream);

/* One reverse step of the discrete adjoint of rsfde_step (no counterpart in
 * the paper; derived from M u^k = u^{k-1} + dt mask f(u^{k-1}) with M
 * symmetric, Corollary 2.1 / Lemma 2.3):
 *   mu       = M^{-1} lam_cur                      (same preconditioned GMRES)
 *   dk[0]   += < mu, (I (x) A_x/kx) u_cur >         (dL/dkx contribution)
 *   dk[1]   += < mu, (A_y/ky (x) I) u_cur >         (dL/dky contribution)
 *   dk[2]   += < mu, (A_z/kz (x) I (x) I) u_cur >   (3-D plans: dL/dkz)
 *   lam_prev = mu + dt * mask * f'(u_prev) * mu
 * u_prev = u^{k-1}, u_cur = u^k, lam_cur = dL/du^k; dk_dev is a device array of
 * two doubles (three for a 3-D plan) accumulated in place.  mu_guess (may be NULL: zero guess) is an
 * initial guess for mu and receives mu on exit when not NULL.
 * lam_prev must not alias lam_cur.  Errors: as rsfde_step. */
int rsfde_adjoint_step(rsfde_plan plan, const double* u_prev, const double* u_cur,
                       const double* lam_cur, int32_t f_kind, const rsfde_solver_opts* opts,
                       double* lam_prev, double* mu_guess, double* dk_dev, rsfde_stats* stats,
                       void* stream);

/* Batched independent solves on one GPU (finite-difference directions,
 * parameter sweeps, ensembles of initial fields).  The paper solves one
 * system per time step; a batch runs `count` such steps (the step of
 * rsfde_step for each member) in lockstep: every FFT pass and every streaming
 * Krylov kernel is launched once for all members still iterating (the members
 * are a grid dimension of each launch), and the host takes one convergence
 * decision per inner step for the whole batch.  Members share the grid,
 * alpha1, alpha2, the mask, eta and dt; each has its own kx, ky, vectors and
 * Krylov state.  The solver is the one-vector flexible GMRES of rsfde_step
 * (right preconditioning, two Gram-Schmidt passes unless opts->reorth = -1,
 * stop when ||b - M x||_2 <= tol ||b||_2, FP64 or FP32 preconditioner).
 *   count        : members, 1 .. 32 (EUNSUPPORTED above)
 *   kx, ky       : host arrays of count coefficients, >= 0
 *   other inputs : as rsfde_setup; n1 + 1 and n2 + 1 must be powers of two
 *                  (EUNSUPPORTED otherwise)
 * The batch owns one region of device memory per member (about
 * (2 max_restart + 6) n1 n2 doubles plus the preconditioner intermediates)
 * and count HostStatus records of pinned memory.
 * Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED. */
typedef struct rsfde_batch_s* rsfde_batch;
int rsfde_batch_setup(rsfde_batch* out, const rsfde_grid* grid, double alpha1, double alpha2,
                      int32_t count, const double* kx, const double* ky,
                      const uint8_t* mask_dev, double eta, double dt, int32_t max_restart,
                      void* stream);
/* New kx, ky for every member (host arrays of count).  Errors: EINVAL, EHIP. */
int rsfde_batch_set_coeffs(rsfde_batch batch, const double* kx, const double* ky);
/* y_m = M_m x_m for every member m: x, y are device arrays [count][n2][n1]
 * (member after member) that must not overlap.  Errors: EINVAL, EHIP. */
int rsfde_batch_matvec(rsfde_batch batch, const double* x, double* y, void* stream);
/* z_m = P_hat_m^{-1} r_m for every member (FP64 or FP32 internals;
 * EUNSUPPORTED for BF16).  Layout as rsfde_batch_matvec. */
int rsfde_batch_precond_apply(rsfde_batch batch, const double* r, double* z, int32_t precision,
                              void* stream);
/* One implicit time step of every member (rsfde_step semantics per member):
 * u_prev, u_prev2 (NULL at the first step), u_next are device arrays
 * [count][n2][n1]; u_next must not alias u_prev.  stats: NULL or count
 * entries, one per member.  opts: restart up to the batch's max_restart,
 * precond RSFDE_PRECOND_TAU, side RSFDE_RIGHT, sstep 0 or 1 (EUNSUPPORTED
 * otherwise).  Returns RSFDE_OK when every member converged, else the first
 * member's failure code (each member's own code is in its stats entry; the
 * other members' results are valid). */
int rsfde_batch_step(rsfde_batch batch, const double* u_prev, const double* u_prev2,
                     int32_t f_kind, const rsfde_solver_opts* opts, double* u_next,
                     rsfde_stats* stats, void* stream);
int rsfde_batch_destroy(rsfde_batch batch);

/* Advance an ensemble of independent plans (finite-difference directions,
 * parameter sweeps, several initial fields: batched solves) by m
 * implicit steps each (rsfde_step semantics: initial guess 2u^{k-1} - u^{k-2},
 * f_kind, opts), concurrently: one host thread per plan, each enqueueing on
 * streams[i] (or that plan's set-up stream when streams is NULL).  Members
 * overlap on the GPU when their streams differ, which keeps small grids from
 * leaving most compute units idle.
 *   plans  : count distinct plans (on the same device)
 *   u0     : count device vectors [n2][n1] of the matching plan (read only)
 *   u_out  : count device vectors receiving u^m (may alias neither u0 nor work)
 *   work   : 2*count device vectors (scratch for the time levels)
 *   stats  : NULL or count entries: iterations summed over the member's steps,
 *            status of its last step
 * Returns RSFDE_OK or the first member's error (every member runs to its end
 * or first error).  Errors: EINVAL, ENOTCONV, ENONFINITE, EHIP. */
int rsfde_march_ensemble(int32_t count, const rsfde_plan* plans, const double* const* u0,
                         int32_t m, int32_t f_kind, const rsfde_solver_opts* opts,
                         double* const* u_out, double* const* work, rsfde_stats* stats,
                         void* const* streams);

/* Kernel timing (measurement support, not part of the method).
 * rsfde_profile(plan, 1) starts bracketing every kernel the plan launches with
 * a pair of HIP events on the launch stream, tagged with the kernel family and
 * its algorithmic byte count (each operand read once, each result written
 * once); rsfde_profile(plan, 0) stops.  rsfde_profile_read waits for the
 * recorded events, fills up to max entries (one per family seen since the
 * last read), sets *count and clears the record.  Errors: EINVAL, EHIP. */
typedef struct {
  char name[24];       /* kernel family, e.g. "multidot", "mv_cols" */
  int64_t launches;    /* launches recorded */
  double total_ms;     /* sum of event-measured durations */
  double bytes;        /* sum of algorithmic bytes of those launches */
} rsfde_kernel_profile;

int rsfde_profile(rsfde_plan plan, int32_t enable);
int rsfde_profile_read(rsfde_plan plan, rsfde_kernel_profile* out, int32_t max, int32_t* count);

/* Release the plan and all of its memory.  NULL is accepted. */
int rsfde_destroy(rsfde_plan plan);

/* Static string for an error code. */
const char* rsfde_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RSFDE_H */
