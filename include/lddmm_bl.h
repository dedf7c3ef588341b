/*
 * lddmm_bl.h - C ABI of the MI355X (gfx950) band-limited PDE-LDDMM library.
 *
 * The library computes the hot path of band-limited Gauss-Newton-Krylov
 * PDE-constrained LDDMM with semi-Lagrangian Runge-Kutta (SL-RK2) integration
 * (M. Hernandez, arXiv 2006.06823):
 *   - the truncated Fourier maps pi (grid -> band) and iota (band -> grid) of
 *     Section 2.2, done as separable dense contractions on the matrix cores;
 *   - the SL-RK2 solves of Table 1 (Section 3.3) for the state, adjoint,
 *     incremental state and incremental adjoint of three variants:
 *       LDDMM_BL_IMAGE_TRANSPORT   original BL PDE-LDDMM (Section 2.3.1),
 *       LDDMM_BL_STATE_EQUATION    BL PDE-LDDMM based on the state equation
 *                                  (Section 2.3.2): m and lambda from the maps
 *                                  phi, psi and the Jacobian J of eq. BLDefState,
 *       LDDMM_BL_DEFORMATION_STATE BL PDE-LDDMM based on the deformation state
 *                                  equation (Section 2.3.3);
 *   - the gradient, the Gauss-Newton Hessian-vector product and the
 *     Gauss-Newton-Krylov driver with PCG preconditioned by L~^{-1}
 *     (Section 2.2, eqs. BLNewton and BLKKT).
 *
 * Conventions (the paper leaves them open; these are the readings used):
 *   - The image domain is the periodic unit torus [0,1)^d with nodes
 *     x = i / N_j.  The L^2 inner product is the grid mean.
 *   - Grid scalars are [N1][N2](..[N3]) in C order (last axis contiguous);
 *     vector fields are component-major [d][N1][N2](..[N3]).
 *   - Band-limited (BL) arrays are [ncomp][K1][K2](..[K3]) coefficients of the
 *     real orthonormal tensor basis: per axis, slot 0 = 1, slots 2k-1 / 2k =
 *     sqrt(2) cos(2 pi k x) / sqrt(2) sin(2 pi k x) for k = 1 .. K_j/2 - 1, and
 *     slot K_j - 1 an always-zero pad.  K_j must be even, K_j - 1 <= N_j, and
 *     N_j >= 3 (K_j/2 - 1) + 1 for alias-free truncated products.
 *   - The energy is 1/2 <L~ v~, v~> + (1/sigma^2) mean((m(1) - I1)^2) with
 *     L~ = (1 + alpha (2 pi)^2 |k|^2)^s (eq. BLEnergy); the velocity is
 *     stationary; time integrals use the trapezoid rule over Nt steps.
 *   - Element type of every device buffer: double for LDDMM_BL_FP64, float
 *     otherwise.  Reductions (objective, dot products, norms, Jacobian) are
 *     accumulated in double on the device.
 *
 * Ownership and ordering: the caller owns every buffer it passes; device
 * buffers are borrowed until the stream has run the call.  The context owns
 * its workspaces (trajectories, departure points, scratch).  Every call runs
 * in order on the stream given at creation and synchronises that stream
 * before it returns, except lddmm_bl_hess_matvec and
 * lddmm_bl_project_noalloc, which only enqueue their work: their results are
 * ready, and their buffers free for other use, once the stream has reached
 * them.  No exception or abort crosses the ABI.
 *
 * Errors: negative status = error (the result is not valid), positive =
 * warning with a valid result.  lddmm_bl_last_error(ctx) gives the text of the
 * last error of a context; lddmm_bl_last_error(NULL) the text of the last error
 * of a call on this thread that has no context (lddmm_bl_create, the batched
 * solve, the network calls).
 */
#ifndef LDDMM_BL_H
#define LDDMM_BL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lddmm_bl_ctx lddmm_bl_ctx;

typedef enum {
  LDDMM_BL_OK = 0,
  LDDMM_BL_E_ARG = -1,        /* invalid argument or size */
  LDDMM_BL_E_OOM = -2,        /* device allocation failed */
  LDDMM_BL_E_HIP = -3,        /* HIP runtime error */
  LDDMM_BL_E_NONFINITE = -4,  /* NaN/Inf in an objective, norm or dot product */
  LDDMM_BL_E_STATE = -5,      /* call order: e.g. adjoint before a state solve at this velocity */
  LDDMM_BL_W_MAXITER = 1,     /* iteration cap reached before the gradient tolerance */
  LDDMM_BL_W_LINESEARCH = 2,  /* Armijo backtracking failed; velocity left unchanged */
  LDDMM_BL_W_NEGCURV = 3      /* reserved: gn_solve records a PCG truncated by non-positive curvature
                                 per iteration in its report (log_negcurv), not in its status */
} lddmm_bl_status;

typedef enum {
  LDDMM_BL_IMAGE_TRANSPORT = 1,   /* original BL PDE-LDDMM, Section 2.3.1 */
  LDDMM_BL_STATE_EQUATION = 2,    /* state equation with the maps phi, psi, J (eq. BLDefState), Section 2.3.2.
                                     Gradient L~v~ + int lambda~ star grad~ m~ with m(t) = I0 o phi(t),
                                     lambda(t) = J(t) lambda(1) o psi(t); Gauss-Newton Hessian with
                                     dlambda(t) = J(t) dlambda(1) o psi(t), dlambda(1) = -(2/sigma^2) dm(1),
                                     dm(1) = -grad P(I0) o phi(1) . iota(du~(1)) (eq. BLIncDefState).  The
                                     nu~ equation is read with right-hand side -v~.  Holds (Nt+1) x 8 grid
                                     fields for m, psi, J and lambda at every node. */
  LDDMM_BL_DEFORMATION_STATE = 3  /* deformation state equation, Section 2.3.3 */
} lddmm_bl_variant;

typedef enum {
  LDDMM_BL_FP64 = 0,   /* every buffer and kernel in double */
  LDDMM_BL_FP32 = 1,   /* float buffers, float contractions, double reductions */
  LDDMM_BL_BF16_DFT = 2 /* float buffers; truncated-DFT contractions on bf16 matrix cores
                          with float accumulation (hi/lo split operands) */
} lddmm_bl_precision;

typedef enum {
  LDDMM_BL_SL_RK2 = 0,    /* semi-Lagrangian Heun steps along the characteristics (Section 3) */
  LDDMM_BL_EULER_RK4 = 1  /* comparator: the deformation-state equations of Section 2.3.3 in Eulerian form,
                             d_t u~ = v~ - D~u~ star v~, d_t rho~ = -div~(rho~ star v~) and their incremental
                             counterparts, integrated by the classical four-stage Runge-Kutta method with exact
                             truncated products (the RK rows of the paper's evaluation, Section 4.3: it needs
                             nt = 25-50 for stability).  The incremental state's D~u~ at half steps is the mean of
                             the two nodes'.  LDDMM_BL_DEFORMATION_STATE only (LDDMM_BL_E_ARG otherwise). */
} lddmm_bl_integrator;

typedef struct {
  int32_t dim;            /* 2 or 3 */
  int32_t n[3];           /* grid N1..Nd (unused entries ignored) */
  int32_t k[3];           /* band K1..Kd, even */
  int32_t nt;             /* SL-RK2 time steps, dt = 1/nt */
  int32_t variant;        /* lddmm_bl_variant */
  double alpha;           /* L = (Id - alpha Laplacian)^s, Section 2.1 */
  int32_t s;
  double sigma2;          /* data weight 1/sigma^2, eq. BLEnergy */
  int32_t precision;      /* lddmm_bl_precision */
  int32_t integrator;     /* lddmm_bl_integrator (0: SL-RK2) */
  int32_t nonstationary;  /* 1: a velocity per time node (Section 1.3; the NSt rows of Tables 3-4) for the
                             image-transport and deformation-state variants with SL-RK2 (LDDMM_BL_E_ARG
                             otherwise).  Velocity-like arrays (v, gradient, dv, H dv, gn_solve's v) are then
                             [nt + 1][d][K..]; the regulariser integrates over the nodes by the trapezoid rule;
                             gradient and Hessian are node fields (the stationary integrands node by node), and
                             PCG and the Armijo test use the node-field product sum_n w_n <a_n, b_n>.  A step's
                             characteristics take the arrival node's velocity at the arrival point and the
                             departure node's at the predicted departure point.  Excludes the batched solve and
                             the low-rank and two-level preconditioners.  0: stationary. */
} lddmm_bl_params;

typedef struct {
  int32_t max_gn;         /* Gauss-Newton iteration cap (Section 4.3: 10) */
  int32_t max_pcg;        /* PCG iteration cap per GN iteration (Section 4.3: 5) */
  double grad_rtol;       /* stop when ||g||_inf <= grad_rtol * reference */
  double grad_ref_inf;    /* reference ||g||_inf; 0 => ||g||_inf at the initial velocity */
  int32_t fixed_iters;    /* 1 => run every cap to the end (no tolerance exits) */
  double energy_target;   /* > 0 => also stop once the objective E <= energy_target (0 = off); used to
                             time how fast a warm-started run reaches a reference run's objective */
  int32_t ml_inner;       /* > 0 => two-level spectral preconditioner (the multi-level preconditioning the
                             Discussion names as the next step): M^-1 r = L~^-1 on the slots above the coarse
                             band Kc = 2 floor(K / 4) and, inside it, ml_inner PCG iterations (from 0, with
                             L~c^-1) on the Gauss-Newton Hessian of the coarse problem (grid N / 2, images
                             restricted by 2^d block means, velocity restricted to Kc) linearised at every GN
                             iteration; the outer iteration is then flexible CG.  Needs even N and a valid
                             coarse band on every axis; excludes precond_Z (LDDMM_BL_E_ARG). 0 = off. */
} lddmm_bl_gn_opts;

#define LDDMM_BL_LOG_MAX 64 /* Gauss-Newton iterations whose decisions the report records */
typedef struct {
  int32_t gn_iters, pcg_iters_total, backtracks, hess_matvecs;
  double E0, E;           /* energy at the start and at the end */
  double mse_rel;         /* ||m(1) - I1||^2 / ||I0 - I1||^2 (Section 5.1.1) */
  double grad_inf_rel;    /* final ||g||_inf / reference */
  double det_min, det_max; /* extrema of det(I - D iota(u~(1))) of the final map (Section 5.1.1, Tables 3-4) */
  double seconds;         /* wall time of the call */
  /* Decisions of Gauss-Newton iteration i < min(gn_iters + 1, LDDMM_BL_LOG_MAX), the discrete
   * branches two implementations can take differently: PCG iterations taken, the PCG exit
   * (0 tolerance or cap, 1 non-positive curvature), and the Armijo backtracks before the
   * accepted step (-1: no step accepted, the solve stopped there). */
  int32_t log_count;
  int32_t log_pcg[LDDMM_BL_LOG_MAX];
  int32_t log_negcurv[LDDMM_BL_LOG_MAX];
  int32_t log_backtracks[LDDMM_BL_LOG_MAX];
} lddmm_bl_gn_report;

/* Create a context for one registration problem.  hip_stream: a hipStream_t
 * (NULL = the default stream).  Allocates every workspace the variant needs. */
lddmm_bl_status lddmm_bl_create(const lddmm_bl_params* params, void* hip_stream, lddmm_bl_ctx** out);
lddmm_bl_status lddmm_bl_destroy(lddmm_bl_ctx* ctx);
const char* lddmm_bl_last_error(const lddmm_bl_ctx* ctx);

/* Source I0 and target I1 (device, grid layout), copied into the context. */
lddmm_bl_status lddmm_bl_set_images(lddmm_bl_ctx* ctx, const void* I0, const void* I1);

/* State solve at velocity v_bl (device, BL [d][K..]): characteristics
 * (Section 3.1), then the state equation (Table 1 row 1 or 3).  Writes the
 * deformed source m(1) (device grid) when m1_or_null is not NULL and
 * {E, regulariser, data term} to E_reg_data (host, may be NULL). */
lddmm_bl_status lddmm_bl_state_solve(lddmm_bl_ctx* ctx, const void* v_bl, void* m1_or_null,
                                     double* E_reg_data);

/* Adjoint solve (Table 1 row 2 or 4) at the velocity of the last state solve
 * and the gradient L~v~ + int (adjoint term) dt (Section 2.3.1 / 2.3.3).
 * grad_bl: device BL [d][K..]; grad_inf (host, may be NULL) = max over grid
 * nodes and components of |iota(g)|.  E_STATE without a prior state solve. */
lddmm_bl_status lddmm_bl_adjoint_solve(lddmm_bl_ctx* ctx, void* grad_bl, double* grad_inf);

/* Gauss-Newton Hessian-vector product at the velocity of the last state solve:
 * incremental state (Table 1 row 5 or 7), final coupling, incremental adjoint
 * (row 6 or 8) and the time integral of the Hessian term.  dv_bl, hdv_bl:
 * device BL [d][K..] (may not alias).  E_STATE without a prior state solve.
 * Enqueued on the context's stream without waiting for it (see the ordering
 * rule above), so back-to-back calls keep the GPU busy; in 3D each call
 * replays a HIP graph captured on the caller's own (dv_bl, hdv_bl) pair (the
 * four most recent pairs are kept). */
lddmm_bl_status lddmm_bl_hess_matvec(lddmm_bl_ctx* ctx, const void* dv_bl, void* hdv_bl);

/* Gauss-Newton-Krylov registration (eqs. BLNewton, BLKKT) starting from
 * v_bl_inout (device BL [d][K..]), which receives the result.  PCG uses
 * L~^{-1}; when precond_Z_or_null is a device array of r BL directions
 * [r][d][K..], the two-level preconditioner L~^{-1} + Z (Z^T H Z)^{-1} Z^T is
 * used instead.  report (host) may be NULL.  When the context holds a state
 * solve at exactly the starting velocity (a state_solve with the same values,
 * no set_images since), that state is reused instead of being solved again.
 * Status: W_LINESEARCH when an Armijo search accepted no step (the velocity is
 * the last accepted one), else W_MAXITER when the GN cap ended a run with
 * tolerance exits before the tolerance was met, else OK. */
lddmm_bl_status lddmm_bl_gn_solve(lddmm_bl_ctx* ctx, const lddmm_bl_gn_opts* opts, void* v_bl_inout,
                                  const void* precond_Z_or_null, int32_t r, lddmm_bl_gn_report* report);

/* Batched Gauss-Newton-Krylov: `count` independent registrations (subjects with
 * their own grid and band, per_subject[i]; FP32 or BF16_DFT precision) run in
 * lockstep, ordered on hip_stream.  The subjects' solves, line-search trials and
 * Hessian matvecs run as parallel branches on up to 8 internal streams forked from
 * and joined back into hip_stream (the matvecs of a PCG iteration as one HIP graph
 * launch); PCG scalars, Armijo decisions and stopping tests stay per subject, each
 * subject running the steps of its own gn_solve.  I0[i], I1[i], v_bl_inout[i]:
 * device buffers of subject i (layouts as above); reports: host array of
 * `count` (may be NULL).  Returns LDDMM_BL_W_LINESEARCH if any subject's line
 * search failed (that subject's velocity is left at its last accepted value).
 * hip_stream must not be NULL (E_ARG): the matvec graph is captured on it.
 * The Gauss-Newton status of each subject follows the rules of lddmm_bl_gn_solve
 * through its report; the returned status is the worst of them. */
lddmm_bl_status lddmm_bl_gn_solve_batched(const lddmm_bl_params* per_subject, int32_t count, const void* const* I0,
                                          const void* const* I1, void* const* v_bl_inout,
                                          const lddmm_bl_gn_opts* opts, void* hip_stream,
                                          lddmm_bl_gn_report* reports);

/* Jacobian determinant det(I - D iota(u~(1))) of phi(1) = id - iota(u~(1))
 * (Sections 2.3.2-2.3.3) at the velocity of the last state solve, evaluated
 * in double.  detmap_or_null: device double grid; minmax: host double[2]. */
lddmm_bl_status lddmm_bl_jacobian(lddmm_bl_ctx* ctx, void* detmap_or_null, double* minmax);

/* Truncated Fourier maps of Section 2.2 on ncomp stacked fields:
 * project: device grid [ncomp][N..] -> device BL [ncomp][K..] (pi);
 * include: device BL [ncomp][K..] -> device grid [ncomp][N..] (iota). */
lddmm_bl_status lddmm_bl_project(lddmm_bl_ctx* ctx, const void* grid, void* bl, int32_t ncomp);
lddmm_bl_status lddmm_bl_include(lddmm_bl_ctx* ctx, const void* bl, void* grid, int32_t ncomp);

/* The projection of lddmm_bl_project for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments, layouts and
 * result, with the reduction's workspace in a static 16 MiB device array of the library instead of
 * the context's buffers.  It calls no hipMalloc / hipFree and does not wait: the kernels are enqueued
 * on the context's stream and the call returns (the result is ready when the stream reaches it).
 * The context's device must be current; the first call on a device looks up that device's copy of the
 * array.  Limits: FP32 contexts on the plane-wise path (not FP64, not split-bf16: LDDMM_BL_E_ARG),
 * ncomp * N0 * K1 * K2 * 4 bytes <= 16 MiB (LDDMM_BL_E_ARG otherwise, with the sizes in the error
 * text).  Every call on one GPU shares that GPU's array: calls that overlap on one GPU (two streams,
 * two threads) race and must be ordered by the caller. */
lddmm_bl_status lddmm_bl_project_noalloc(lddmm_bl_ctx* ctx, const void* grid, void* bl, int32_t ncomp);

/* Internal fields of the last solves, for inspection and parity checks.
 * Copies field `which` at time node `index` into dst (device) and returns the
 * number of elements through count (host).  With dst = NULL only the count is
 * returned.  Grid fields use the grid layout, BL fields the BL layout. */
typedef enum {
  LDDMM_BL_FIELD_VELOCITY = 0,     /* iota(v~) [d][N..] */
  LDDMM_BL_FIELD_DEP_BACKWARD = 1, /* departure displacement X - x for forward-in-time equations, grid units [d][N..] */
  LDDMM_BL_FIELD_DEP_FORWARD = 2,  /* departure displacement for backward-in-time equations [d][N..] */
  LDDMM_BL_FIELD_DIV_V = 3,        /* iota(div~ v~) [N..] */
  LDDMM_BL_FIELD_STATE = 4,        /* image-transport: m at node index [N..]; state-equation and deformation-state:
                                      u~ at node index [d][K..] */
  LDDMM_BL_FIELD_M1 = 5,           /* m(1) [N..] */
  LDDMM_BL_FIELD_ADJOINT0 = 6,     /* image-transport and state-equation: lambda(0) [N..]; deformation-state:
                                      rho~(0) [d][K..] */
  LDDMM_BL_FIELD_INC_STATE = 7,    /* dm~ [K..] or du~ [d][K..] at node index, from the last matvec */
  LDDMM_BL_FIELD_INC_ADJOINT = 8,  /* dlambda~ [K..] (image-transport; state-equation: pi(dlambda(t_n))) or
                                      drho~ [d][K..] at node index, from the last matvec */
  LDDMM_BL_FIELD_INVERSE_STATE = 9,  /* state-equation: nu~ at node index [d][K..] (psi = id - iota(nu~)) */
  LDDMM_BL_FIELD_JACOBIAN_STATE = 10, /* state-equation: J~ = 1 - U~ at node index [K..] */
  LDDMM_BL_FIELD_IMAGE = 11,       /* image-transport and state-equation: m(t_n) at node index [N..] */
  LDDMM_BL_FIELD_ADJOINT_GRID = 12 /* state-equation: lambda(t_n) at node index [N..], from the last adjoint solve */
} lddmm_bl_field;
lddmm_bl_status lddmm_bl_get_field(lddmm_bl_ctx* ctx, int32_t which, int32_t index, void* dst, int64_t* count);

/* Device-side FP64 reductions used by PCG, exposed for checks:
 * dot = sum a_i b_i over n elements of the context's element type. */
lddmm_bl_status lddmm_bl_dot(lddmm_bl_ctx* ctx, const void* a, const void* b, int64_t n, double* dot);

/* Learned warm start and low-rank preconditioner (a small 3D convolutional network
 * trained on registrations the method itself computes; an addition feeding the initial
 * guess and the PCG preconditioner of eqs. BLNewton / BLKKT, Section 2.2).  `levels` 3^3
 * convolutions (padding 1, ReLU; stride 2 except the last) with channels[0..levels-1] on
 * a 2-channel input of in_size^3 voxels (the image pair, [B][2][S][S][S] float), then a
 * 1^3 head to 3 (1 + rank_r) channels, rank_r in 0..16: the predicted velocity (channels
 * 0..2) and rank_r low-rank preconditioner directions (3 channels each).  The head output
 * [B][3 (1 + rank_r)][s][s][s], s = in_size / 2^(levels-1), holds grid samples on the
 * coarse s^3 grid of the unit torus.  Kernels: bf16 matrix-core implicit-GEMM
 * convolutions with float accumulation; float master weights; Adam.
 * forward keeps the activations for backward; backward accumulates parameter
 * gradients (zero_grad clears them); get copies parameters (which = 0) or their
 * gradients (which = 1) to host (nparam floats), set loads parameters from host.
 * save writes the architecture and the float master parameters to a file (an 8-byte
 * tag, int32 levels, channels, in_size, rank_r, [out_size,] int64 nparam, then the
 * parameters; out_size only in files of networks made by lddmm_nn_create_out, under
 * their own tag); load reads such a file into a network of the same architecture
 * (E_ARG on a mismatch or an unreadable file).  Errors of these calls are reported
 * through lddmm_bl_last_error(NULL).
 * lddmm_nn_create_out makes the same network with the output grid out_size^3 instead
 * (the levels take stride 2 while the grid is larger than out_size, then stride 1;
 * out_size = in_size / 2^j for some j < levels, else E_ARG; 0 selects the default
 * schedule): out_size = 32 predicts every coefficient of a 32^3 band. */
typedef struct lddmm_nn_ctx lddmm_nn_ctx;
lddmm_bl_status lddmm_nn_create(int32_t levels, const int32_t* channels, int32_t in_size, int32_t rank_r,
                                uint64_t seed, void* hip_stream, lddmm_nn_ctx** out);
lddmm_bl_status lddmm_nn_create_out(int32_t levels, const int32_t* channels, int32_t in_size, int32_t out_size,
                                    int32_t rank_r, uint64_t seed, void* hip_stream, lddmm_nn_ctx** out);
lddmm_bl_status lddmm_nn_info(lddmm_nn_ctx* ctx, int32_t* out_size, int32_t* out_channels, int64_t* nparam);
lddmm_bl_status lddmm_nn_forward(lddmm_nn_ctx* ctx, const void* in, int32_t B, void* out);
lddmm_bl_status lddmm_nn_backward(lddmm_nn_ctx* ctx, const void* dout, int32_t B);
lddmm_bl_status lddmm_nn_zero_grad(lddmm_nn_ctx* ctx);
lddmm_bl_status lddmm_nn_step(lddmm_nn_ctx* ctx, double lr);
lddmm_bl_status lddmm_nn_get(lddmm_nn_ctx* ctx, int32_t which, void* host_dst);
lddmm_bl_status lddmm_nn_set(lddmm_nn_ctx* ctx, const void* host_src);
lddmm_bl_status lddmm_nn_save(const lddmm_nn_ctx* ctx, const char* path);
lddmm_bl_status lddmm_nn_load(lddmm_nn_ctx* ctx, const char* path);
lddmm_bl_status lddmm_nn_destroy(lddmm_nn_ctx* ctx);

/* Input and output maps of the warm-start network (all device float, on the network's stream).
 * pool_pair: box average of an image pair I0, I1 [n0][n1][n2] (each n_j a multiple of in_size) into
 *   one network input slot [2][in_size^3] (I0 in channel 0).
 * velocity: network output [B][3 (1 + r)][s^3] -> band-limited coefficients
 *   v_bl [B][1 + r][3][k0][k1][k2] (the velocity, then the r directions): the projection of
 *   Section 2.2 onto the s-point band (frequencies |m| <= s/2 - 1, i.e. real slots 0 .. s-2 per
 *   axis), zero in every other slot.  Requires even k_j >= s - 1.
 * loss: mean over the batch of the squared V-norm error sum_a L~(a) (v_pred - v_target)_a^2 of the
 *   velocity channels, L~ = (1 + alpha (2 pi)^2 |m|^2)^s (Section 2.1), accumulated in double;
 *   v_target [B][3][K]; writes d loss / d output to dout_or_null ([B][3 (1 + r)][s^3], zero on
 *   the direction channels) when it is not NULL. */
lddmm_bl_status lddmm_nn_pool_pair(lddmm_nn_ctx* ctx, const void* I0, const void* I1, const int32_t* n,
                                   void* in_slot);
lddmm_bl_status lddmm_nn_velocity(lddmm_nn_ctx* ctx, const void* out, int32_t B, const int32_t* k, void* v_bl);
lddmm_bl_status lddmm_nn_loss(lddmm_nn_ctx* ctx, const void* out, const void* v_target, int32_t B,
                              const int32_t* k, double alpha, int32_t s, void* dout_or_null, double* loss);

/* Per-kernel timing for measurement tools (process-wide).  While enabled,
 * every kernel launch of the library is bracketed with HIP events on its
 * stream and its algorithmic bytes and flops are recorded (enabling clears
 * old records).  lddmm_bl_profile_read(NULL, 0) collects the records into a
 * text table, one line per kernel: name, launches, total ms, algorithmic
 * bytes, flops (tab separated), and returns the buffer size it needs;
 * lddmm_bl_profile_read(buf, len) then copies the table into buf. */
lddmm_bl_status lddmm_bl_profile_enable(int32_t on);
int64_t lddmm_bl_profile_read(char* buf, int64_t len);

/* Autotuner cache (process-wide).  The interpolation kernels of a context pick one of
 * lddmm_bl_tune_candidates("brick") workgroup tiles per grid shape and staging width
 * (fields staged together: 1, 2 or 3), timing every candidate when the first context of
 * that shape is created, under the keys "brick:<n0>x<n1>x<n2>:gs<w>".  Contexts whose
 * truncated DFT does not run the plane-wise path (LDDMM_BL_BF16_DFT) also pick one of
 * lddmm_bl_tune_candidates("dft") workgroup caps (256, 512, 768, 1024, 1536, 2048) for each
 * first-axis contraction shape at creation, under keys "dft:<kernel>:M<m>:L<l>:C<c>"; a
 * shape first met later (or inside graph capture) takes the kernel's default cap.
 * tune_get returns the cached choice of a key, or -1 if none.  tune_set fixes the choice
 * of a key before a context of that shape is created (choice in [0, candidates), or -1
 * to forget it so that the next context times the candidates again); it returns
 * LDDMM_BL_E_ARG for an unknown key family or a choice out of range.  A key's choice is
 * read at every launch, so a context created before a tune_set follows it too; calls that
 * overlap launches on other threads race. */
int32_t lddmm_bl_tune_candidates(const char* family);
int32_t lddmm_bl_tune_get(const char* key);
lddmm_bl_status lddmm_bl_tune_set(const char* key, int32_t choice);
/* The cache as text, one "key=choice" line per key: lddmm_bl_tune_table(NULL, 0) takes a
 * snapshot and returns the bytes needed (with the terminating zero, -1 on failure), then
 * lddmm_bl_tune_table(buf, len) copies it into buf (truncated to len - 1 characters) and
 * returns the characters copied. */
int64_t lddmm_bl_tune_table(char* buf, int64_t len);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_BL_H */
