/*
 * dgmf.h - C ABI of the MI355X matrix-free DG operator library (libdgmf.so).
 *
 * Operators of the discontinuous Galerkin discretisation of Sec. 3.2 on
 * periodic Cartesian hexahedral meshes with tensor-product Lagrange bases on
 * Legendre-Gauss-Lobatto (LGL) nodes of degree k and Gauss quadrature, and
 * the preconditioned CG solver, the inverse mass matrix, the Helmholtz
 * operator, the projection-step operator and its inverse-mass-preconditioned
 * solve, and the h-multigrid level transfers and V-cycle of Sec. 3.3.  All compute runs
 * in HIP kernels for gfx950.
 *
 * Mesh and layout (every entry point)
 *   - elements per direction n_el[d], box edge length[d]; element size
 *     h_d = length[d] / n_el[d]; periodic in all three directions.
 *   - element e = ex + Nx*(ey + Ny*ez); n = k+1; local node i = a + n*(b + n*c),
 *     a the x index (fastest); node (a,b,c) sits at reference point
 *     (xi_a, xi_b, xi_c) of the LGL nodes xi on [0, 1].
 *   - scalar field: [N_el][n^3]; vector field: [3][N_el][n^3] (component major).
 *   - element arrays are contiguous; 256-byte aligned device pointers are
 *     recommended (any 8-byte (f64) / 4-byte (f32) alignment is accepted).
 *
 * Ownership and synchronisation
 *   - every array pointer is a caller-owned DEVICE pointer, except where a
 *     parameter says "host".  The library owns only its own small caches
 *     (1D tables, solver work vectors).
 *   - apply / vjp / divergence / gradient / inverse mass / Helmholtz /
 *     projection / transfer calls are
 *     asynchronous on `hip_stream`
 *     (a hipStream_t; NULL = the default stream).  dg_cg_solve blocks until
 *     it returns, and so does dg_mass_pcg_solve.
 *   - outputs are overwritten, never accumulated.  Inputs and outputs must
 *     not overlap (DG_ERR_ALIAS); dg_apply_inverse_mass alone also accepts
 *     dst == src (in place).
 *
 * Errors
 *   - 0 = DG_OK.  Negative codes are hard errors: nothing was launched and
 *     outputs are untouched.  Positive codes are soft solver failures: x holds
 *     the last iterate and the report is filled.  No C++ exception crosses the
 *     ABI.  dg_last_error() gives a per-thread message for the last failure.
 */
#ifndef DGMF_H
#define DGMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DG_OK = 0,
  DG_ERR_INVALID_ARG = -1,   /* null pointer, bad size, non-finite parameter */
  DG_ERR_UNSUPPORTED = -2,   /* degree or quadrature count without a kernel   */
  DG_ERR_ALIAS = -3,         /* an output overlaps an input                   */
  DG_ERR_HIP = -4,           /* a HIP runtime call failed                     */
  DG_NOT_CONVERGED = 1,      /* CG hit max_iter before the tolerance          */
  DG_ERR_BREAKDOWN = 2       /* CG met p.Ap <= 0, or a NaN/Inf residual       */
};

typedef enum { DG_F64 = 0, DG_F32 = 1 } dg_dtype;

/* Operator descriptor.  All fields are used exactly as given. */
typedef struct {
  int32_t degree;          /* k, 1..11 (n = k+1 LGL nodes per direction)            */
  int32_t n_el[3];         /* elements per direction, each >= 1                      */
  double  length[3];       /* box edge per direction, > 0 (2*pi for [-pi, pi]^3)     */
  int32_t n_q;             /* 1D Gauss points; 0 = default: k+1 for the Laplace and
                              divergence forms, floor(3k/2)+1 (the 3/2 rule of
                              Sec. 3.2) for the convective form                      */
  double  penalty_factor;  /* SIPG penalty tau = penalty_factor*(k+1)^2/h_d on faces
                              normal to d (the paper gives no formula; 1 is usual)  */
  double  scale;           /* multiplies the Laplace form (nu for the viscous v_h)  */
  int32_t n_comp;          /* Laplace: 1 (pressure) or 3 (velocity, per component)  */
  double  lf_factor;       /* coefficient of the Lax-Friedrichs jump term; the
                              paper's c_h has 1 (no factor 1/2)                     */
} dg_op_desc;

/*
 * SIPG negative Laplacian l_h (Sec. 3.2, weak form of l_h; v_h is `scale`
 * times it per component):
 *   dst_i = scale * [ (grad phi_i, grad u)_K
 *                     + sum_faces ( -1/2 (grad phi_i . n)(u- - u+)
 *                                   -1/2 phi_i (grad u- + grad u+) . n
 *                                   + tau phi_i (u- - u+) ) ]
 * with n the outward normal of the element that owns phi_i.
 *   src, dst: [n_comp][N_el][n^3] of `dtype` (double or float).
 * Degrees 1..11; n_q in k+1..32 (k+1 already integrates exactly on these
 * affine cells, Sec. 3.2; fewer points return DG_ERR_UNSUPPORTED).
 * The operator is symmetric, so it is also its own vector-Jacobian product.
 */
int dg_apply_laplace(const dg_op_desc* desc, dg_dtype dtype, const void* src, void* dst,
                     void* hip_stream);

/*
 * Convective term c_h with the local Lax-Friedrichs flux (Sec. 3.2, weak form
 * of c_h, F_c(u) = u (x) u):
 *   r_{c,i} = -(d_j phi_i, u_c u_j)_K
 *             + sum_faces (phi_i, 1/2 (u-_c (u-.n) + u+_c (u+.n))
 *                                 + lf_factor * max(|u-.n|, |u+.n|) (u-_c - u+_c))
 * with the maximum taken pointwise at each face quadrature point.
 *   u, r: [3][N_el][n^3] of `dtype`.  n_q must be 0 or floor(3k/2)+1.
 */
int dg_apply_convective(const dg_op_desc* desc, dg_dtype dtype, const void* u, void* r,
                        void* hip_stream);

/*
 * Vector-Jacobian product of dg_apply_convective: grad_u = J(u)^T w.
 * Cell part g_j = -(phi, sum_m u_m d_m w_j + sum_i u_i d_j w_i).  Face part
 * (each element from its own side, no atomics): (phi, sum_i (w-_i - w+_i)
 * dF*_i/du-_j).  At kinks of the max the derivative takes 1/2 from each side
 * on exact ties |u-.n| = |u+.n|, and sign(0) = 0.
 *   u, w, grad_u: [3][N_el][n^3] of `dtype`; grad_u must not overlap u or w.
 * Built for k <= 11 in FP64 and FP32; higher degrees return
 * DG_ERR_UNSUPPORTED.
 */
int dg_vjp_convective(const dg_op_desc* desc, dg_dtype dtype, const void* u, const void* w,
                      void* grad_u, void* hip_stream);

/*
 * Helmholtz operator of the viscous step (Sec. 3.3: gamma_0/dt M + nu L,
 * solved with the inverse mass as preconditioner): dst = mass_factor M src +
 * scale L src, with L the SIPG form of dg_apply_laplace (desc->scale = nu,
 * penalty, n_q as there) and M the mass matrix of the DG space
 * (dg_apply_inverse_mass).  mass_factor must be finite and >= 0.
 *   src, dst: [n_comp][N_el][n^3] of `dtype`, must not overlap.
 */
int dg_apply_helmholtz(const dg_op_desc* desc, dg_dtype dtype, double mass_factor, const void* src, void* dst,
                       void* hip_stream);

/*
 * Operator of the projection step (Sec. 3.3, (M + A_D + A_C) u, with the
 * divergence and continuity penalty terms of Sec. 3.2):
 *   y = (v, u)_K + (div v, tau_D div u)_K + sum_faces (v . n, {tau_C} [[u]] . n)
 * with [[u]] = u^- - u^+, {tau_C} the mean of the two elements' values and n
 * the own element's outward normal; k+1 Gauss points per direction (n_q must
 * be 0 or k+1, else DG_ERR_UNSUPPORTED); desc->n_comp must be 3.
 *   u, y: [3][N_el][n^3] of `dtype`; tau_d, tau_c: [N_el] of `dtype`, the
 *   element values of the two penalty parameters (the paper builds them from
 *   the extrapolated velocity, h/(k+1) and the time step).  y must not
 *   overlap u, tau_d or tau_c.
 */
int dg_apply_projection(const dg_op_desc* desc, dg_dtype dtype, const void* u, const void* tau_d,
                        const void* tau_c, void* y, void* hip_stream);

/*
 * Pressure gradient g_h with central flux (Sec. 3.2, weak form of g_h), the
 * pressure term of the projection step's right-hand side without its
 * dt/gamma_0 factor:
 *   y_j,i = -(d_j phi_i, p)_K + sum over the faces normal to e_j of
 *           n_j (phi_i, 1/2 (p- + p+))
 * On the periodic mesh it is minus the transpose of dg_apply_divergence.
 *   p: [N_el][n^3], y: [3][N_el][n^3] of `dtype`; y must not overlap p.
 *   Uses n_q (default k+1).
 */
int dg_apply_gradient(const dg_op_desc* desc, dg_dtype dtype, const void* p, void* y, void* hip_stream);

/*
 * Level transfers of the h-multigrid hierarchy (Sec. 3.3: geometric multigrid
 * with matrix-free transfers).  `coarse` describes the coarse mesh; the fine
 * mesh has 2*n_el[d] elements per direction on the same box, same degree.
 * dg_prolongate embeds the coarse DG space in the fine one: the fine element
 * with child index (cx, cy, cz) of its parent gets the parent's polynomial
 * at its nodes, u_f = (P_cx (x) P_cy (x) P_cz) u_parent with
 * P_c[i][a] = l_a((xi_i + c)/2).  dg_restrict applies the transpose, summing
 * the eight children of each coarse element.
 *   uc, rc: [n_comp][N_el][n^3] on the coarse mesh; uf, rf: [n_comp][8 N_el][n^3]
 *   on the fine mesh (element numbering of the fine mesh); `dtype`; n_comp
 *   1 or 3; src and dst must not overlap.
 */
int dg_prolongate(const dg_op_desc* coarse, dg_dtype dtype, const void* uc, void* uf, void* hip_stream);
int dg_restrict(const dg_op_desc* coarse, dg_dtype dtype, const void* rf, void* rc, void* hip_stream);

/*
 * Velocity divergence d_h with central flux (Sec. 3.2, weak form of d_h), the
 * right-hand side of the pressure Poisson step without its -gamma_0/dt factor:
 *   b_i = -(grad phi_i, u)_K + sum_faces (phi_i, 1/2 (u- + u+) . n)
 *   u: [3][N_el][n^3], b: [N_el][n^3] of `dtype`.  Uses n_q (default k+1).
 */
int dg_apply_divergence(const dg_op_desc* desc, dg_dtype dtype, const void* u, void* b,
                        void* hip_stream);

/*
 * Inverse mass matrix of the DG space (Sec. 3.3: block-diagonal, one dense
 * block per element, inverted element by element by sum factorisation; used
 * there for the convective step and as the preconditioner of the projection
 * and Helmholtz equations): dst = M^-1 src with M_ij = (phi_i, phi_j), Gauss
 * quadrature with k+1 points per direction (exact).  n_comp (1 or 3) blocks
 * per element, layout as dg_apply_laplace.
 *   src, dst: [n_comp][N_el][n^3] of `dtype`.  dst may equal src (in place);
 *   any other overlap returns DG_ERR_ALIAS.  n_q < k+1 returns
 *   DG_ERR_UNSUPPORTED (the under-integrated mass matrix is singular).
 */
int dg_apply_inverse_mass(const dg_op_desc* desc, dg_dtype dtype, const void* src, void* dst,
                          void* hip_stream);

enum { DG_PC_JACOBI_F64 = 0, DG_PC_CHEB_F32 = 1 };

typedef struct {
  int32_t precond;       /* DG_PC_JACOBI_F64: z = D^-1 r in double;
                            DG_PC_CHEB_F32: Chebyshev smoother of D^-1 A in float
                            (Sec. 3.3: degree 5, smoothing range 20), started at 0  */
  int32_t cheb_degree;   /* error-polynomial degree; degree-1 float applies per call */
  double  cheb_range;    /* lambda_min = lambda_max / cheb_range                     */
  double  rtol, atol;    /* stop when ||r||_2 <= max(rtol*||b||_2, atol)             */
  int32_t max_iter;
  int32_t project_mean;  /* 1: keep r and z at zero coefficient mean (periodic)     */
} dg_cg_opts;

typedef struct {
  int32_t iterations;    /* CG iterations done                                       */
  int32_t matvec_f64;    /* double-precision operator applications launched          */
  int32_t matvec_f32;    /* single-precision operator applications launched          */
                         /* (iterations run in batches between host checks of the    */
                         /*  residual; a batch may end with a few no-op iterations   */
                         /*  after convergence, counted here and in seconds_solve)   */
  double  rel_res;       /* recursive ||r||/||b|| at exit                             */
  double  true_rel_res;  /* ||b - A x||/||b|| recomputed in double at exit           */
  double  lambda_max;    /* estimate of the largest eigenvalue of D^-1 A (Chebyshev) */
  double  seconds_solve; /* wall time of the iteration (setup excluded)              */
  double  seconds_setup; /* diagonal, eigenvalue estimate, work vectors              */
} dg_cg_report;

/*
 * Solve A x = b with the SIPG form of dg_apply_laplace (n_comp must be 1) by
 * preconditioned CG (Sec. 3.3) in double precision: residuals, dot products
 * and the updates of x, r and p stay in double on the GPU.  DG_PC_JACOBI_F64
 * uses the standard beta; with DG_PC_CHEB_F32 the preconditioner runs
 * single-precision operator applies and beta is the flexible
 * (Polak-Ribiere) one, r+.(z+ - z)/(r.z).
 *   b: [N_el][n^3] double (device); x: [N_el][n^3] double (device), initial
 *   guess in, solution out; report: host pointer, may be NULL.
 * Returns DG_OK, DG_NOT_CONVERGED or DG_ERR_BREAKDOWN (x holds the last
 * iterate), or a negative error.  Blocks the calling thread.
 */
int dg_cg_solve(const dg_op_desc* desc, const dg_cg_opts* opts, const double* b, double* x,
                dg_cg_report* report, void* hip_stream);

/*
 * dg_cg_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, arguments, results and errors, but it calls no hipMalloc,
 * hipHostMalloc, hipFree or allocating library routine.  Every piece of device
 * memory beyond b and x (six double and five float work vectors, partial
 * sums, the iteration state, the diagonal, the operator tables) is carved
 * from one static device array of 64 MiB per GPU, held from the library's
 * load until the process ends; host reads go through stack buffers (the
 * small operator plan and tables are built in ordinary host memory).
 * Limit: 68 bytes per DoF plus a fixed part under 1 MiB, about 0.97e6 DoFs
 * (k = 7 on 12^3 elements fits); a larger problem returns
 * DG_ERR_INVALID_ARG before touching the GPU.  Calls on one GPU share the
 * array and its contents persist between calls (each call initialises what
 * it reads); the library serialises calls from the threads of one process,
 * and the call blocks until the solve has finished, so calls never overlap
 * inside one process.
 */
int dg_cg_solve_noalloc(const dg_op_desc* desc, const dg_cg_opts* opts, const double* b, double* x,
                        dg_cg_report* report, void* hip_stream);

/*
 * Divergence and gradient between the mixed-order spaces of the paper's
 * solver (Sec. 3.2: velocity of tensor degree k, pressure of degree k-1,
 * inf-sup stable), central fluxes, k+1 Gauss points (exact on affine cells):
 *   dg_apply_divergence_mixed: b_i = d_h(q_i, u) = -(grad q_i, u)_K +
 *     (q_i, {{u}}.n)_dK for the degree-(k-1) basis q_i;
 *     u: [3][N_el][(k+1)^3], b: [N_el][k^3];
 *   dg_apply_gradient_mixed: y_j,i = g_h(phi_i e_j, p) = -(d_j phi_i, p)_K +
 *     (phi_i n_j, {{p}})_dK for the degree-k basis phi_i;
 *     p: [N_el][k^3], y: [3][N_el][(k+1)^3].
 * desc: degree = k (2..11), the mesh; n_q 0 or k+1; n_comp, scale, penalty
 * and lf_factor unused.  dtype DG_F64 or DG_F32; device pointers, the output
 * must not overlap the input.  Asynchronous on hip_stream.  On a periodic
 * mesh the gradient is minus the transpose of the divergence.
 */
int dg_apply_divergence_mixed(const dg_op_desc* desc, dg_dtype dtype, const void* u, void* b, void* hip_stream);
int dg_apply_gradient_mixed(const dg_op_desc* desc, dg_dtype dtype, const void* p, void* y, void* hip_stream);

/*
 * Taylor-Green diagnostics of a velocity field (Sec. 4.2):
 *   out[0] = e_k = (1/V) int 1/2 u.u,  out[1] = eps = (nu/V) int grad u : grad u
 * (gradients element by element, k+1 Gauss points: exact), V the box volume.
 * u: [3][N_el][(k+1)^3] doubles (device); out: 2 doubles (host).  Blocks.
 */
int dg_tgv_diagnostics(const dg_op_desc* desc, const double* u, double nu, double* out, void* hip_stream);

typedef struct {
  int32_t order;          /* 1: BDF1 (the start-up step, u_nm1 unused); 2: BDF2 */
  double  dt;             /* time step */
  double  nu;             /* kinematic viscosity */
  double  zeta_d;         /* divergence penalty factor (the paper: 1) */
  double  zeta_c;         /* continuity penalty factor (the paper: 1) */
  double  rtol_pressure;  /* relative CG tolerances of the three solves (the paper: 1e-6) */
  double  rtol_projection;
  double  rtol_viscous;
  double  atol_pressure;  /* absolute tolerance of the pressure solve (the paper: 1e-12) */
  int32_t max_iter;       /* iteration limit of each solve */
  int32_t pressure_precond;   /* DG_STEP_PC_GMG_F32 (0, the default) or DG_STEP_PC_CHEB_F32 */
} dg_step_opts;

/* Preconditioners of the pressure CG of dg_dual_splitting_step: one FP32
 * V-cycle of dg_gmg_cg_solve per iteration (Sec. 3.3, the paper's choice) on
 * as many levels as the element counts allow (all halved while even with
 * halves of at least 2, at most 5 levels), with the library's level bounds;
 * or the FP32 Chebyshev(5) smoother of dg_cg_solve. */
enum { DG_STEP_PC_GMG_F32 = 0, DG_STEP_PC_CHEB_F32 = 1 };

typedef struct {
  int32_t it_pressure, it_projection, it_viscous;   /* CG iterations of the three solves */
  double  kinetic_energy;   /* e_k of u_np1 */
  double  dissipation;      /* eps of u_np1 (nu from opts) */
  double  seconds;          /* wall time of the call */
} dg_step_report;

/*
 * One time step of the dual splitting scheme (Sec. 3.1; matrix form of
 * Sec. 3.3) on the periodic mesh of desc, in double precision, no body force:
 *   convective step  U^ = (sum_i alpha_i U^{n-i} - dt M^-1 sum_i beta_i C(U^{n-i})) / gamma_0
 *   pressure step    L P = -(gamma_0/dt) D U^        (degree k-1; FP64 CG with the FP32
 *                                                     V-cycle or Chebyshev(5)
 *                                                     preconditioner, opts->pressure_precond)
 *   projection step  (M + A_D + A_C) U^^ = M U^ - (dt/gamma_0) G P   (inverse-mass PCG)
 *   viscous step     (gamma_0/dt M + nu L) U^{n+1} = (gamma_0/dt) M U^^  (inverse-mass PCG)
 * BDF1: gamma_0 = 1, alpha = 1, beta = 1; BDF2: gamma_0 = 3/2,
 * alpha = (2, -1/2), beta = (2, -1).  C is the convective form of
 * dg_apply_convective (lf_factor from desc), D and G those of the mixed-order
 * calls above, L the SIPG form (penalty_factor from desc) at degree k-1 for
 * the pressure and k for the velocity, A_D and A_C those of
 * dg_apply_projection with tau_D = zeta_d |u_ex|_e h/(k+1) dt and
 * tau_C = zeta_c |u_ex|_e dt per element, u_ex = sum_i beta_i U^{n-i},
 * |u_ex|_e its element-averaged magnitude, h = (element volume)^(1/3).
 *   desc: velocity degree k (2..11), the mesh; n_q 0; scale and n_comp unused.
 *   u_n, u_nm1 (order 2), u_np1: [3][N_el][(k+1)^3] doubles (device);
 *   p: [N_el][k^3] doubles (device): in, the pressure solve's initial guess
 *   (e.g. the previous pressure); out, P^{n+1} (zero coefficient mean).
 *   u_np1 and p must not overlap each other or the inputs.
 * The library keeps five velocity-sized work vectors per GPU.  Returns
 * DG_OK, a negative error, or DG_NOT_CONVERGED / DG_ERR_BREAKDOWN of the
 * solve that failed (u_np1 then does not hold the step's result).  Blocks.
 */
int dg_dual_splitting_step(const dg_op_desc* desc, const dg_step_opts* opts, const double* u_n,
                           const double* u_nm1, double* u_np1, double* p, dg_step_report* report,
                           void* hip_stream);

/*
 * The same step with the convective term kept across steps (Sec. 3.1: the
 * BDF2 extrapolation uses C(U^n) and C(U^{n-1}), and C(U^{n-1}) is the
 * previous step's C(U^n)):
 *   conv_nm1: C(u_nm1) as returned by the previous call in its conv_n, or
 *             NULL (then computed); ignored for order 1;
 *   conv_n:   out, C(u_n) (the convective form of dg_apply_convective,
 *             before the inverse mass), for the next call, or NULL;
 *   both [3][N_el][(k+1)^3] doubles (device), overlapping neither each
 *   other nor the velocities or p (DG_ERR_ALIAS).  With conv_nm1 from the
 *   previous call the result is bit-identical to dg_dual_splitting_step;
 *   a conv_nm1 that is not C(u_nm1) gives a different (wrong) step.
 */
int dg_dual_splitting_step_conv(const dg_op_desc* desc, const dg_step_opts* opts, const double* u_n,
                                const double* u_nm1, const double* conv_nm1, double* conv_n, double* u_np1,
                                double* p, dg_step_report* report, void* hip_stream);

enum { DG_OP_HELMHOLTZ = 0, DG_OP_PROJECTION = 1 };

/*
 * Solve the Helmholtz equation of the viscous step or the projection equation
 * by CG preconditioned with the inverse mass matrix (Sec. 3.3: the block-
 * diagonal mass is inverted element by element at the cost of a diagonal
 * scaling and serves as the preconditioner of both steps), in double
 * precision, k+1 Gauss points (n_q must be 0 or k+1):
 *   DG_OP_HELMHOLTZ:  (mass_factor M + L) x = b, L the form of
 *                     dg_apply_laplace (scale, penalty_factor from desc),
 *                     mass_factor > 0, n_comp 1 or 3; tau_d, tau_c unused;
 *   DG_OP_PROJECTION: (M + A_D + A_C) x = b, the operator of
 *                     dg_apply_projection; n_comp = 3; tau_d, tau_c: [N_el]
 *                     doubles (device); mass_factor unused.
 *   b, x: [n_comp][N_el][n^3] doubles (device); x: initial guess in,
 *   solution out; must not overlap b, tau_d or tau_c.  Stops when
 *   ||r||_2 <= rtol ||b||_2 (recursive residual); report: host pointer, may
 *   be NULL (then no true residual is computed; lambda_max and matvec_f32
 *   are 0).
 * The iteration scalars stay on the device; the host checks the state once
 * per batch of iterations (report->matvec_f64 counts the no-op iterations
 * that may end the last batch).
 * Returns DG_OK, DG_NOT_CONVERGED or DG_ERR_BREAKDOWN (x holds the last
 * iterate), or a negative error.  Blocks the calling thread; runs on
 * hip_stream.
 */
int dg_mass_pcg_solve(const dg_op_desc* desc, int32_t op, double mass_factor, const double* tau_d,
                      const double* tau_c, const double* b, double* x, double rtol, int32_t max_iter,
                      dg_cg_report* report, void* hip_stream);

/*
 * One V-cycle of geometric multigrid for the SIPG form of dg_apply_laplace
 * (Sec. 3.3: the pressure Poisson preconditioner; Chebyshev smoothing of
 * D^-1 A on [lambda_max/smoothing_range, lambda_max], the same degree before
 * and after the coarse-grid correction, a Chebyshev method with
 * coarse_degree steps on the coarsest level, matrix-free transfers of
 * dg_prolongate / dg_restrict), all in the precision `dtype`:
 *   z = V r,  level l = the mesh coarsened l times by two per direction
 *   (re-discretised SIPG operator and diagonal), l = 0..levels-1.
 * Post-smoothing smooths the residual equation from zero.
 *   desc: the finest mesh, n_comp = 1, element counts divisible by
 *   2^(levels-1); lambda_max: host array of `levels` eigenvalue bounds of
 *   D_l^-1 A_l (level diagonals and Chebyshev coefficients are rounded to
 *   FP32 for DG_F32), or NULL: then each level's bound is the one
 *   dg_cg_solve estimates for the Chebyshev preconditioner (1.1 x the largest
 *   Ritz value of 25 Lanczos steps, kept per operator); dtype: DG_F64 or
 *   DG_F32; r, z: [N_el][n^3] values of that type (device), must not overlap.
 * Allocates its level vectors, blocks until the cycle has run.
 */
int dg_gmg_vcycle(const dg_op_desc* desc, int32_t levels, int32_t degree, double smoothing_range,
                  int32_t coarse_degree, const double* lambda_max, int32_t dtype, const void* r, void* z,
                  void* hip_stream);

/*
 * Solve A x = b with the SIPG form (n_comp = 1, periodic: b and the
 * iterates are taken at zero coefficient mean) by FP64 CG preconditioned with
 * one V-cycle per iteration (the cycle of dg_gmg_vcycle: degree,
 * smoothing_range and coarse_degree as there; Sec. 3.3 uses 5, 20 and a
 * coarse Chebyshev solve of degree 10), flexible beta.
 *   lambda_max: host array of `levels` bounds as for dg_gmg_vcycle, or NULL
 *   (estimated per level as there);
 *   cycle_dtype: DG_F64 (the cycle of dg_gmg_vcycle) or DG_F32 (the cycle in
 *   single precision: the residual rounded to FP32 on entry, the cycle's
 *   output entering the FP64 direction update, the CG itself in FP64 as
 *   Sec. 3.3 splits the work);
 *   b, x: [N_el][n^3] doubles (device), x: initial guess in, solution out;
 *   stops when |r| <= rtol |b - mean(b)|; report: host pointer, may be NULL;
 *   its matvec_f64 / matvec_f32 count the outer FP64 applies and every
 *   level apply of the cycles (all levels) by precision, lambda_max the
 *   finest level's bound.  The iteration scalars stay on the device; the
 *   host reads the state once per batch of up to four iterations, so the
 *   counts include the cycle after the last iteration and any iterations
 *   queued after convergence (which leave x unchanged).
 * Returns DG_OK, DG_NOT_CONVERGED or DG_ERR_BREAKDOWN, or a negative error.
 * Blocks the calling thread.
 */
int dg_gmg_cg_solve(const dg_op_desc* desc, int32_t levels, int32_t degree, double smoothing_range,
                    int32_t coarse_degree, const double* lambda_max, int32_t cycle_dtype, const double* b, double* x,
                    double rtol, int32_t max_iter, dg_cg_report* report, void* hip_stream);

/*
 * diag(A) of the SIPG form on one element (identical on every element of a
 * uniform periodic mesh with at least 2 elements per direction): host array of
 * n^3 doubles.  Setup for the Jacobi and Chebyshev preconditioners (Sec. 3.3:
 * the diagonal is precomputed in the setup phase).
 */
int dg_laplace_diagonal(const dg_op_desc* desc, double* diag_host);

/* The k+1 LGL nodes of degree k on [0, 1] (Sec. 3.2), into a host array. */
int dg_lgl_nodes(int32_t degree, double* nodes_host);

const char* dg_error_string(int code);
/* Message of the last failing call on this thread ("" if none). */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGMF_H */
