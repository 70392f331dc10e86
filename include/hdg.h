/*
 * hdg.h - C ABI of the MI355X (gfx950) library for the statically condensed,
 * matrix-free hybridizable discontinuous Galerkin (HDG) operator of
 * Huismann, Stiller & Froehlich, "Linearizing the hybridizable discontinuous
 * Galerkin method: A linearly scaling operator" (arXiv:2007.11891).
 *
 * Problem (paper, equation (helmholtz_equation)):
 *     lambda u - laplace u = f  in the box [0, sum h_1] x [0, sum h_2] x [0, sum h_3],
 *     u = g_D on the Dirichlet sides (all six unless hdg_create_ex names
 *     Neumann sides), n . grad u = g_N on the Neumann sides (outward n),
 * discretised on a Cartesian mesh of n1 x n2 x n3 cuboids with per-axis
 * widths, Lagrange polynomials of degree p on Gauss-Lobatto-Legendre (GLL)
 * points (lumped GLL mass matrix), penalty tau_{i,e} = 2 tau_hat / h_{i,e}
 * (section "LDG operator structure in three dimensions").  After static
 * condensation only the face trace u~ remains: K u~ = F (equation
 * (hdg_system)), K = sum_e Q_e^T K_e Q_e with K_e the Schur complement of
 * equation (hdg_operator).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers: arguments documented "device" are device pointers of the GPU the
 * context was created on; "host" pointers are read during the call only.
 * The caller owns every buffer it passes; the library never frees or keeps
 * them.  Buffers must not overlap unless stated.
 *
 * Streams: all device work is enqueued on the stream given to hdg_create
 * (a hipStream_t passed as void*, NULL = the null stream), in call order.
 * Entry points that need a host decision (the solvers) synchronise that
 * stream; all others return without waiting.
 *
 * Errors: every entry point returns hdg_status.  Arguments are validated
 * before any work is enqueued; on error nothing is enqueued and
 * hdg_last_error() returns a message (thread-local, valid until the next
 * call on the same thread).  HIP failures return HDG_EHIP.
 *
 * Layouts (n_p = p + 1):
 *   Volume vectors (length n_vol = n1 n2 n3 n_p^3): element
 *     e = i + n1 (j + n2 k), then node q1 + n_p (q2 + n_p q3), q1 fastest
 *     (the paper's Kronecker ordering, equation (tp_definition)).
 *   Trace vectors: the unknowns ("free" part, length n_free) are the
 *     interior faces normal to x1, then x2, then x3, followed by the faces
 *     of the Neumann sides; then the "tail" (length n_all - n_free): the
 *     faces of the Dirichlet sides (g_D), then the g_N block, which holds
 *     n . grad u at the nodes of each Neumann face in the order of those
 *     faces in the free part.  Interior faces of axis a sit on planes
 *     m = 1..n_a-1 and are ordered with x1 fastest over (plane, element
 *     indices of the two other axes):
 *         a=0: (m-1) + (n1-1)(j + n2 k)
 *         a=1: i + n1((m-1) + (n2-1) k)
 *         a=2: i + n1(j + n2 (m-1))
 *     Sides are numbered k = 2a + s (s = 0 the plane m = 0, s = 1 the plane
 *     m = n_a) and come in increasing k, each ordered t_b + n_b t_c over the
 *     two tangential element indices (b < c): the Neumann sides in the free
 *     part, the Dirichlet sides in the tail.  With no Neumann side the free
 *     part is the interior faces and the tail every boundary face.
 *     Within a face: n_p x n_p nodes, q_b + n_p q_c (lower axis fastest).
 *   Bases of trace vectors: HDG_BASIS_NODAL holds nodal values (u~) or
 *     nodal residuals; HDG_BASIS_EIGEN holds the transformed unknowns of the
 *     section "Product factorization of the HDG operator":
 *     u^ = (S^T M x S^T M) u~ per face, and F^ = (S^T x S^T) F for residuals,
 *     where S^T M S = I, S^T L S = Lambda (equation
 *     (generalized_eigenvalue_decomposition)).  K^ = T^T K T, T = S x S.
 */
#ifndef HDG_H
#define HDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_ctx hdg_ctx;

typedef enum {
  HDG_OK = 0,
  HDG_EINVAL = -1,       /* invalid argument */
  HDG_EHIP = -2,         /* a HIP runtime call failed */
  HDG_ENOMEM = -3,       /* device or host allocation failed */
  HDG_ENOCONV = -4,      /* solver stopped at maxit; info is filled */
  HDG_EUNSUPPORTED = -5  /* valid request the library does not implement */
} hdg_status;

typedef enum { HDG_F64 = 0, HDG_F32 = 1 } hdg_dtype;
typedef enum { HDG_BASIS_NODAL = 0, HDG_BASIS_EIGEN = 1 } hdg_basis;

/* Face transforms of the section "Product factorization of the HDG operator"
 * and of the transformed solver listing, applied per face as A x A:
 *   HDG_TO_EIGEN_UNKNOWN   u^ = (S^T M x S^T M) u~
 *   HDG_TO_EIGEN_RESIDUAL  F^ = (S^T x S^T) F
 *   HDG_TO_NODAL_UNKNOWN   u~ = (S x S) u^
 *   HDG_TO_NODAL_RESIDUAL  F  = (M S x M S) F^                              */
typedef enum {
  HDG_TO_EIGEN_UNKNOWN = 0,
  HDG_TO_EIGEN_RESIDUAL = 1,
  HDG_TO_NODAL_UNKNOWN = 2,
  HDG_TO_NODAL_RESIDUAL = 3
} hdg_transform;

/* Solver options.  By default the CG runs on K^_ff in the eigen-face basis
 * with the diagonal (Jacobi) preconditioner of K^ (the paper's HDG-trans
 * solver, section "Summary of solution method"); x0 = 0.  precond 0, 2 and 3
 * select the paper's other solvers of that section, which run the CG in the
 * nodal trace basis with the operator applied through the face transforms
 * (FP64 only, textbook form; `variant` and `mixed` do not apply):
 *   0  HDG-unprec: no preconditioner;
 *   2  HDG-diag: the main diagonal of the inverse face blocks of K_ff
 *      (section "Preconditioners");
 *   3  HDG-block: the inverse face blocks of K_ff (algorithm
 *      "Block_Preconditioner"), applied as (S x S) diag(1/y) (S^T x S^T).
 * For them rtol and rel_res refer to the nodal basis (||F||_2). */
typedef struct {
  double rtol;        /* stop when ||r||_2 <= rtol ||F^||_2 (eigen basis)   */
  int maxit;          /* iteration cap (FP64 CG, or per inner FP32 solve)   */
  int precond;        /* 0: none, 1: Jacobi in the eigen basis (default),
                         2: nodal diagonal, 3: nodal face blocks (above)   */
  int mixed;          /* 0: FP64 CG; 1: FP32 CG with FP64 residual replacement
                         (reliable updates: the FP32 CG keeps its search
                         direction across replacements); precond 1 only,
                         else HDG_EUNSUPPORTED                               */
  double inner_rtol;  /* mixed: residual reduction of each FP32 segment between
                         two FP64 residual replacements (values below 1e-4
                         are raised to 1e-4)                                 */
  int max_outer;      /* mixed: cap on defect-correction steps              */
  int check_every;    /* iterations per host convergence poll (>= 1)        */
  int variant;        /* CG form: 0 one kernel per iteration (Chronopoulos-
                         Gear form of the same PCG: one reduction point per
                         iteration); 1 textbook PCG, an element kernel and a
                         vector update kernel per iteration; 2 textbook PCG
                         with the pencil element kernel (blocks march up x3,
                         the faces between consecutive elements carried in
                         registers; x updated in the element launch) and a
                         vector update kernel; -1 the context's choice
                         (hdg_autotune, or by mesh size).  Mixed precision
                         runs its FP32 inner CG in form 1 whatever this is */
  int guess;          /* 0: CG from x0 = 0; 1: the unknowns passed in (u_free
                         of hdg_solve, the free part of trace in
                         hdg_solve_forcing) are the initial guess, e.g. from
                         hdg_hybridize (section "Summary of solution method").
                         The CG then solves for the correction from the
                         residual F - K x0 with the stopping test unchanged
                         (||r|| <= rtol ||F||, in the solver's basis); iters
                         counts the correction's iterations, 0 when x0 already
                         passes.  2: the same start, stopped when
                         ||r|| <= rtol ||r_0|| (the paper's protocol for its
                         test case: the initial residual reduced by rtol).
                         rel_res is relative to ||F|| in every case.
                         hdg_adjoint ignores it.                            */
} hdg_solve_opts;

typedef struct {
  int iters;          /* CG iterations (FP64, or FP32 inner summed)          */
  int outer_iters;    /* defect-correction steps (mixed), else 0            */
  double rel_res;     /* final ||F^ - K^ u^||_2 / ||F^||_2, recomputed in FP64 */
  double rhs_norm;    /* ||F^||_2                                            */
  double t_ms;        /* wall time of the solve on the stream               */
} hdg_solve_info;

/* Fill *opts with defaults: rtol 1e-10, maxit 20000, Jacobi, FP64,
 * inner_rtol 1e-2, max_outer 12, check_every 25, variant -1. */
void hdg_default_opts(hdg_solve_opts* opts);

/* Create a context for one mesh (paper section "LDG operator structure in
 * three dimensions": Cartesian cuboids, per-axis widths, tau_{i,e}).
 *   n_elem      host int[3], elements per axis, each >= 1
 *   h1, h2, h3  host double arrays of n_elem[0..2] widths, each > 0
 *   p           polynomial degree, 1 <= p <= 16
 *   tau_hat     penalty scale tau_hat > 0
 *   lambda_host host double[n1 n2 n3] per-element lambda >= 0, or NULL to
 *               use lambda_const >= 0 everywhere
 *   stream      hipStream_t (as void*) used for all work of this context
 * The one-time setup (GLL points, 1D matrices, the generalized
 * eigendecomposition S, Lambda and B_S of equation (hdgbs), and the
 * diagonal of K^) runs in FP64: the 1D part on the host, the diagonal on the
 * GPU.  On success *out owns device memory until hdg_destroy. */
hdg_status hdg_create(const int n_elem[3], const double* h1, const double* h2,
                      const double* h3, int p, double tau_hat,
                      const double* lambda_host, double lambda_const,
                      void* stream, hdg_ctx** out);

/* hdg_create with Neumann sides and the choice of mass matrix.
 * neumann_sides (0..63): bit 2a + s makes side s of axis a (s = 0:
 * x_{a+1} = 0, s = 1: x_{a+1} = sum h_{a+1}) a Neumann side (equation
 * (neumann_flux)), n . grad u = g_N, whose trace is unknown; the others stay
 * Dirichlet.  The layout of trace vectors follows (see "Layouts" above).
 * All six sides Neumann with lambda = 0 everywhere is rejected (HDG_EINVAL):
 * the condensed operator is then singular.
 * exact_mass (0 or 1): 1 takes the exact mass matrix M_ij = int phi_i phi_j
 * of the GLL Lagrange basis instead of the lumped diag(w) (the paper's
 * remark that lumping keeps the face terms diagonal): S, Lambda, B_S follow
 * from it, and in the eigen basis the face term of each axis is the 2 x 2
 * matrix G + C^T M^-1 C, which couples the two opposite faces of an element
 * (at the same tangential index).  The forcing, recovery and transforms use
 * the same M.
 * hdg_create is this call with 0, 0.  Batched solves stay Dirichlet with the
 * lumped mass. */
hdg_status hdg_create_ex(const int n_elem[3], const double* h1, const double* h2,
                         const double* h3, int p, double tau_hat,
                         const double* lambda_host, double lambda_const,
                         int neumann_sides, int exact_mass, void* stream, hdg_ctx** out);

/* Release the context and its device memory (synchronises its stream). */
hdg_status hdg_destroy(hdg_ctx* ctx);

/* Thread-local message of the last failed call. */
const char* hdg_last_error(void);

/* Vector lengths: trace unknowns (free), whole trace (free part, g_D block
 * and g_N block), volume nodes. */
/* The same lengths for a mesh, degree and set of Neumann sides without a
 * context (host-only, touches no GPU; arguments as in hdg_create_ex). */
hdg_status hdg_layout(const int n_elem[3], int p, int neumann_sides, int64_t* n_free,
                      int64_t* n_all, int64_t* n_vol);

hdg_status hdg_sizes(const hdg_ctx* ctx, int64_t* n_free, int64_t* n_all,
                     int64_t* n_vol);

/* Replace the per-element lambda field (device double[n_elem], >= 0, not
 * checked on the device) and rebuild the diagonal preconditioner.  With
 * every side Neumann, lambda must stay > 0 somewhere (not checked here;
 * lambda = 0 everywhere makes the operator singular). */
hdg_status hdg_set_lambda(hdg_ctx* ctx, const double* lambda_dev);

/* Host-only: the 1D tables the context uses, for degree p and tau_hat
 * (equations (element_matrices), (generalized_eigenvalue_decomposition),
 * (hdgbs)).  Each output is a host array, row-major, or NULL to skip:
 * x, w [n_p] GLL points and weights; D [n_p*n_p] with D_ij = int phi_i phi_j';
 * S [n_p*n_p] (S_ij = S[i*n_p+j], columns = eigenvectors); Lam [n_p]
 * ascending; BS [n_p*2] with BS[k*2+s]; H [1], the diagonal value of
 * G + C^T M^-1 C.  Touches no GPU. */
hdg_status hdg_tables(int p, double tau_hat, double* x, double* w, double* D,
                      double* S, double* Lam, double* BS, double* H);

/* Physical coordinates of the volume nodes (device double[n_vol*3], xyz
 * interleaved) and of the trace nodes (device double[n_all*3]; the g_N block
 * repeats the nodes of its Neumann faces); either may be NULL.  Synchronous
 * (computed on the host, copied on the stream). */
hdg_status hdg_coords(hdg_ctx* ctx, double* vol_xyz, double* trace_xyz);

/* Place the mesh corner at origin[3] (host doubles, finite; default 0, 0, 0)
 * for hdg_coords.  The condensed operator, the right-hand side and the
 * recovery depend on the element widths only (the metric factors of the
 * transformed element operator, paper section "Product factorization of the
 * HDG operator"), so the origin moves nothing but the coordinates a caller
 * evaluates f and the boundary data at. */
hdg_status hdg_set_origin(hdg_ctx* ctx, const double origin[3]);

/* y = K_ff x (paper: Alg. "HDG_Op_3D", nodal basis, or the transformed
 * Alg. with product factorization, eigen basis), on the free trace:
 * x, y device arrays of n_free values of type dtype, not overlapping.
 * Boundary (Dirichlet) unknowns are zero.  The element loop applies the
 * transformed operator; in the nodal basis the face transforms of the
 * product-factorization section wrap it. */
hdg_status hdg_apply(hdg_ctx* ctx, const void* x, void* y, hdg_dtype dtype,
                     hdg_basis basis);

/* hdg_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same y = K_ff x with the same arguments and kernels, but its per-face
 * element contributions (and, in the nodal basis, the transformed input) sit
 * in one file-scope device array of 48 MiB per GPU instead of context memory,
 * so the call itself allocates nothing.  The array is held on each GPU the
 * library runs on until the process ends; its device address is looked up
 * once per device, at the first call on that device (the current device must
 * be the context's).  Limit: 2 (eigen basis) or 3 (nodal basis) vectors of
 * n_free values of dtype, each rounded up to 256 bytes, must fit in 48 MiB
 * (n_free up to about 3.1M in FP64, eigen basis); larger sizes return
 * HDG_EINVAL and launch nothing.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other contexts, other
 * threads) race.  Nothing in the array needs clearing between calls. */
hdg_status hdg_apply_noalloc(hdg_ctx* ctx, const void* x, void* y, hdg_dtype dtype,
                             hdg_basis basis);

/* Per-face transform (see hdg_transform) of n_faces consecutive faces
 * (n_faces * n_p^2 FP64 values, device; n_faces <= n_all / n_p^2); in == out
 * is allowed. */
hdg_status hdg_face_transform(hdg_ctx* ctx, hdg_transform kind,
                              const double* in, double* out, int64_t n_faces);

/* Right-hand side of the condensed system with the Dirichlet lift,
 *     F_f = F(f)_f - K_fD g_D + g_N,f,   F(f)_e = -R_e^T A_e^-1 [M_e f_e; 0]
 * (derived from eliminating u, q in the element system; the printed solver
 * listing has the opposite sign), evaluated by fast diagonalisation:
 * F^_e = -B^_e^T D_Z^-1 (S_e^T M_e f_e - B^_e u^_D,e).  g_N,f is the face
 * integral of mu g_N on the Neumann faces (the flux row of the element
 * system, equation (ldg_element_operator)): (h_b h_c / 4) (M x M) g_N.
 *   f        device double[n_vol] nodal forcing
 *   trace    device double[n_all] nodal trace; only the tail (g_D and g_N)
 *            is read; NULL means g_D = 0 and g_N = 0
 *   F_free   device double[n_free] output in the requested basis */
hdg_status hdg_rhs(hdg_ctx* ctx, const double* f, const double* trace,
                   double* F_free, hdg_basis basis);

/* Solve K_ff u_f = F_f by preconditioned CG in the eigen-face basis
 * (transformed solver listing: transform, pCG on K^, transform back).
 *   F_free   device double[n_free], nodal residual basis
 *   u_free   device double[n_free], output nodal trace unknowns (input: the
 *            initial guess when opts->guess = 1)
 * Returns HDG_ENOCONV (info filled, u_free = last iterate) when the cap is
 * reached.  Synchronises the stream.  opts NULL = defaults. */
hdg_status hdg_solve(hdg_ctx* ctx, const double* F_free, double* u_free,
                     const hdg_solve_opts* opts, hdg_solve_info* info);

/* Whole solution process for forcing f and boundary data: RHS, CG in the
 * eigen basis, back transform, recovery of u per element.
 *   f        device double[n_vol]
 *   trace    device double[n_all] in: tail = g_D and g_N (nodal), and with
 *            opts->guess = 1 the free part = initial guess; out: free part =
 *            nodal solution trace (tail unchanged)
 *   u_vol    device double[n_vol] output, or NULL to skip the recovery */
hdg_status hdg_solve_forcing(hdg_ctx* ctx, const double* f, double* trace,
                             double* u_vol, const hdg_solve_opts* opts,
                             hdg_solve_info* info);

/* Recovery of u in every element from the trace (paper: last loop of the
 * primal solver listing, sign read from the element system):
 *     u_e = S_e D_Z^-1 (S_e^T M_e f_e - B^_e u^_e)
 *   f      device double[n_vol];  trace device double[n_all] nodal (free
 *   part and g_D tail);  u_vol device double[n_vol] output. */
hdg_status hdg_reconstruct(hdg_ctx* ctx, const double* f, const double* trace,
                           double* u_vol);

/* Initial guess of the trace from a volume field (paper, section "Summary
 * of solution method": q = grad u by differentiation, then the flux of
 * equation (fluxu) on every face):
 *     u~ = (tau+ u+ + tau- u-) / (tau+ + tau-) - (q+.n+ + q-.n-) / (tau+ + tau-)
 * with tau = 2 tau_hat / h_a of the element on either side and q.n the
 * derivative of the element polynomial along the outward normal at the face
 * node.  On a Neumann face the outside brings tau- = 0 and q-.n- = -g_N:
 * u~ = u+ - (q+.n+ - g_N) / tau+.
 *   u_vol       device double[n_vol] volume field (e.g. the last time step)
 *   trace       device double[n_all]; only the g_N block is read; NULL
 *               means g_N = 0
 *   trace_free  device double[n_free] output, nodal (may be the free part of
 *               trace) */
hdg_status hdg_hybridize(hdg_ctx* ctx, const double* u_vol, const double* trace,
                         double* trace_free);

/* Adjoint of u(lambda, f) for a scalar loss J(u) (not in the paper; derived
 * from equation (hdg_operator_factorized) and the recovery formula).  Given
 * the forward solution (trace, u not needed) and r = dJ/du:
 *     j^ = -B^^T D_Z^-1 S_e^T r_e,   K^_ff mu^ = j^ (same CG),
 *     a_E = D_Z^-1 (S_e^T r_e - B^_e mu^_e),  u_E = D_Z^-1 (S_e^T M_e f_e - B^_e u^_e)
 *     dJ/dlambda_e = -d0_e sum a_E u_E,   dJ/df_e = M_e S_e a_E.
 *   f, trace   the forward inputs/solution (device, as in hdg_solve_forcing)
 *   dJdu       device double[n_vol]
 *   dJdlambda  device double[n_elem] output
 *   dJdf       device double[n_vol] output
 * The adjoint CG uses opts (NULL = defaults); info describes it. */
hdg_status hdg_adjoint(hdg_ctx* ctx, const double* f, const double* trace,
                       const double* dJdu, double* dJdlambda, double* dJdf,
                       const hdg_solve_opts* opts, hdg_solve_info* info);

/* Tile shape of the element kernels: elements per work unit = the largest
 * count that fits 256 threads and 60 KB of LDS, shifted right by `variant`
 * (0, 1 or 2).  Synchronises the stream; invalidates captured CG graphs. */
hdg_status hdg_set_tile(hdg_ctx* ctx, int variant);

/* Segment length of the pencil CG form (hdg_solve_opts.variant 2): its
 * element blocks march up x3 through `ks` elements each (1 <= ks <= n3);
 * 0 restores the automatic choice (whole columns when the rows of the mesh
 * give enough blocks, shorter segments otherwise).  Synchronises the stream;
 * invalidates captured CG graphs.  HDG_EINVAL for ks < 0 or ks > n3. */
hdg_status hdg_set_cg_segment(hdg_ctx* ctx, int ks);

/* Autotuner: times one FP64 CG iteration in each of the three CG forms (see
 * hdg_solve_opts.variant; the pencil form with its automatic segment length
 * and with 16, 8, 4 and 2 elements per segment) for every tile variant on
 * this context's mesh (`reps` launches each, HIP events on the context
 * stream), keeps the fastest as the context's tile shape, CG form and
 * segment length, returns the tile variant in *chosen and, in times_ms (host
 * double[3] or NULL), the best time of each tile variant.  Synchronises the
 * stream. */
hdg_status hdg_autotune(hdg_ctx* ctx, int reps, int* chosen, double* times_ms);

/* Current tile shape: *variant (0..2), *elems_per_unit (elements of one
 * work unit), *threads_per_unit (threads of one FP64 work unit, a multiple
 * of 64), and the context's CG form *cg_variant (0, 1 or 2); any pointer may
 * be NULL.  Host-only, no GPU work. */
hdg_status hdg_tile_shape(const hdg_ctx* ctx, int* variant, int* elems_per_unit,
                          int* threads_per_unit, int* cg_variant);

/* Diagonal of K^_ff (eigen basis), device double[n_free] output. */
hdg_status hdg_diagonal(hdg_ctx* ctx, double* diag_free);

/* Kernels and kernel sequences that hdg_time_kernel can time. */
typedef enum {
  HDG_TIME_ELEM_APPLY_F64 = 0,     /* eigen-basis element kernel alone (x -> qa, qb) */
  HDG_TIME_ELEM_APPLY_F32 = 1,
  HDG_TIME_CG2_ITER_F64 = 2,       /* two-kernel CG iteration: fused apply + update */
  HDG_TIME_CG2_ITER_F32 = 3,
  HDG_TIME_CG2_APPLY_F64 = 4,      /* the fused CG apply alone */
  HDG_TIME_CG2_UPDATE_F64 = 5,     /* the CG update alone */
  HDG_TIME_CG2_APPLY_F32 = 6,
  HDG_TIME_CG2_UPDATE_F32 = 7,
  HDG_TIME_COPY_F64 = 8,           /* plain copy x -> y (reference traffic) */
  HDG_TIME_CG1_ITER_F64 = 9,       /* one-kernel CG iteration (solver variant 0) */
  HDG_TIME_CG1_ITER_F32 = 10,
  HDG_TIME_CG1_GRAPH_F64 = 11,     /* the same, replayed from one captured graph */
  HDG_TIME_CG1_GRAPH_F32 = 12,
  HDG_TIME_NODAL_UNPREC_F64 = 13,  /* one nodal-basis CG iteration, precond 0 */
  HDG_TIME_NODAL_DIAG_F64 = 14,    /* precond 2 */
  HDG_TIME_NODAL_BLOCK_F64 = 15,   /* precond 3 */
  HDG_TIME_APPLY_F64 = 16,         /* eigen-basis hdg_apply as it runs: element kernel + sum */
  HDG_TIME_APPLY_F32 = 17,
  HDG_TIME_PENCIL_ITER_F64 = 18,   /* pencil CG iteration (solver variant 2): update + element */
  HDG_TIME_PENCIL_ITER_F32 = 19
} hdg_timed_kernel;

/* Timing helper: launch the kernel or kernel sequence `which`
 * (hdg_timed_kernel) `reps` times back-to-back on the context stream between
 * two HIP events and return the mean time per launch in *ms.  The CG ids
 * run one iteration of a solve that never converges (x as its right-hand
 * side); the graph ids capture reps (rounded up to even) iterations once and
 * time one replay, as the solver runs them.  x, y device buffers of n_free
 * values of the matching type (x read; y written by HDG_TIME_COPY_F64 and
 * HDG_TIME_APPLY_*, which need a y distinct from x).  Unknown ids give
 * HDG_EINVAL.  Synchronises. */
hdg_status hdg_time_kernel(hdg_ctx* ctx, int which, const void* x, void* y,
                           int reps, double* ms);

/* ------------------------------------------------------------------------
 * Batched solves.  Many independent problems, each the paper's Dirichlet
 * problem on the unit cube [0,1]^3 with a uniform n1 x n2 x n3 mesh
 * (h_a = 1 / n_a), its own degree p and constant lambda, homogeneous
 * Dirichlet data, solved together by the HDG-trans CG (section "Summary of
 * solution method") in one persistent launch: all problems iterate in
 * lockstep phases, each keeps its own reductions and stops on its own
 * convergence test.  The right-hand sides, the persistent CG and the
 * recovery are replayed from one captured HIP graph (if the runtime cannot
 * capture the cooperative launch, the graph is split around it).
 *
 * Layout: the per-problem vectors of the single-problem entry points are
 * concatenated in problem order (volume vectors by n_vol, free traces by
 * n_free, see hdg_batch_sizes).
 * ---------------------------------------------------------------------- */
typedef struct hdg_batch hdg_batch;

typedef struct {
  int iters;          /* CG iterations of this problem                         */
  int status;         /* HDG_OK, HDG_ENOCONV (iteration cap) or HDG_EHIP
                         (CG breakdown: p.q <= 0 or not finite)                */
  double rel_res;     /* ||r||_2 / ||F^||_2 of the CG recursion (eigen basis)  */
} hdg_batch_result;

/* Create a batch of `count` >= 1 problems.
 *   n_elem3   host int[count][3], elements per axis, each in [1, 4096]
 *   p         host int[count], degrees in [1, 10]
 *   lambda    host double[count], lambda >= 0 per problem
 *   tau_hat   penalty scale > 0 (all problems)
 *   stream    hipStream_t (as void*) for all work of the batch
 * Tile variants start at 0 for every degree.  *out owns device memory until
 * hdg_batch_destroy.  HDG_EINVAL also when a problem's free trace holds
 * 2^28 values or more (the element pass addresses it with 32-bit byte
 * offsets). */
hdg_status hdg_batch_create(int count, const int* n_elem3, const int* p, const double* lambda,
                            double tau_hat, void* stream, hdg_batch** out);
hdg_status hdg_batch_destroy(hdg_batch* batch);

/* Per-problem sizes (host int64[count] each, either may be NULL) and the
 * totals (host int64, may be NULL). */
hdg_status hdg_batch_sizes(const hdg_batch* batch, int64_t* n_free, int64_t* n_vol,
                           int64_t* total_free, int64_t* total_vol);

/* Tile variant (as in hdg_set_tile) of the work units of every problem of
 * degree p (p = 0: all degrees); hdg_batch_tiles reports the current
 * variant per degree into host int[17] (index p, -1 where no problem has
 * that degree).  set_tile synchronises the stream and drops the graph. */
hdg_status hdg_batch_set_tile(hdg_batch* batch, int p, int variant);
hdg_status hdg_batch_tiles(const hdg_batch* batch, int* variants);

/* CG form of the persistent kernel: 0 (default) two phases per iteration
 * (element pass with the fused p update and the previous iteration's x
 * step, then a vector update of z), two grid barriers; 1 one element pass
 * per iteration with the Chronopoulos-Gear
 * recurrences of the single-problem one-kernel CG (the same PCG iterates in
 * exact arithmetic), one barrier; 2 two phases on the pencil march of the
 * single-problem pencil form (whole columns along x3 per work item, the
 * faces between consecutive elements of a column summed in registers, x
 * updated in the element pass), two barriers.  set_form synchronises the
 * stream, drops the graph and rebuilds the work schedule (each form has its
 * own grid, work item and cost model); hdg_batch_form reports the current
 * form. */
hdg_status hdg_batch_set_form(hdg_batch* batch, int form);
hdg_status hdg_batch_form(const hdg_batch* batch, int* form);

/* Autotuner: for each CG form, starting from variant 0 everywhere, tries
 * variants 1 and 2 for one degree at a time (degrees by decreasing share of
 * the work) and keeps a change when the persistent CG, timed over `iters`
 * iterations (best of `reps` launches), gets faster; the faster form with
 * its tiles stays.  variants: host int[17] or NULL, as in hdg_batch_tiles.
 * Synchronises the stream. */
hdg_status hdg_batch_autotune(hdg_batch* batch, int iters, int reps, int* variants);

/* Mean time in *ms of one persistent CG launch of exactly `iters`
 * iterations for every problem (right-hand side of ones in the eigen basis,
 * no convergence test), over `reps` launches timed with HIP events on the
 * batch stream.  Overwrites the batch's internal right-hand side.
 * Synchronises the stream. */
hdg_status hdg_batch_time_cg(hdg_batch* batch, int iters, int reps, double* ms);

/* Solve every problem: F from f (nodal, as hdg_rhs with zero Dirichlet
 * data), CG in the eigen basis to opts->rtol (FP64 only; opts->mixed must
 * be 0; NULL = defaults), then the nodal trace and, when u_vol is not NULL,
 * the volume solution (as hdg_reconstruct).
 *   f          device double[total_vol]
 *   trace_free device double[total_free] output (the boundary trace is 0)
 *   u_vol      device double[total_vol] output or NULL
 *   results    host hdg_batch_result[count] output or NULL
 *   t_ms       host double output or NULL: GPU time of the whole pipeline
 * Returns HDG_ENOCONV if any problem stopped unconverged, HDG_EHIP if the
 * persistent kernel reported a failed grid barrier.  Synchronises. */
hdg_status hdg_batch_solve_forcing(hdg_batch* batch, const double* f, double* trace_free,
                                   double* u_vol, const hdg_solve_opts* opts,
                                   hdg_batch_result* results, double* t_ms);

#ifdef __cplusplus
}
#endif

#endif /* HDG_H */
