/*
 * bem.h - C ABI of the MI355X boundary-element library for the multiple-domain
 * Helmholtz transmission problem (PMCHWT formulation, Galerkin P1 triangles).
 *
 * Problem statement (paper, section "Model formulation", eq. model): an
 * unbounded exterior Omega^0 (wavenumber k0, density rho0) containing n
 * disjoint bounded domains Omega^j (k_j, rho_j), each touching only the
 * exterior (no triple points).  The unknowns are the exterior Cauchy traces
 * u_j = (gamma_D^{j,+} p_tot, gamma_N^{j,+} p_tot) on every boundary
 * (eq. Form2_matrix_format_p2); the system is
 *   (A^j_{k0} + D_j^-1 A^j_{kj} D_j) u_j + sum_{i != j} A^{ji}_{k0} u_i = gamma^{j,+} p_inc
 * (eq. Form2_calderon_sys_simp3) with the Calderon operator A = [[-K, V], [W, K']]
 * and D_j = diag(1, rho_j/rho_0) (eq. Form1_BCs).  It is discretised with
 * continuous piecewise-linear test and trial functions (eq. Galerkin_disc_lhs,
 * eq. Galerkin_disc_rhs1).  Quadrature: 6-point degree-4 rule per triangle for
 * pairs of triangles sharing no vertex, Sauter-Schwab rules (Gauss-Legendre
 * order ss_order per dimension) for coincident, edge- and vertex-adjacent
 * pairs of the same boundary.
 *
 * Unknown ordering: domain by domain, [u_D^1 (n_v^1), u_N^1 (n_v^1),
 * u_D^2, u_N^2, ...]; u_D entries follow the domain's vertex order.  Several
 * right-hand sides are stored RHS-major: vector r starts at r * n_unknowns.
 *
 * Complex numbers are two doubles (re, im).  Every function returns a status;
 * on a non-OK status, bem_last_error() gives a message (per thread).
 * Handles are not thread-safe: serialise calls on one handle.
 */
#ifndef BEM_MI355X_H
#define BEM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BEM_OK = 0,
    BEM_WARN_NOT_CONVERGED = 1,   /* GMRES stopped at max_iter; best iterate returned */
    BEM_ERR_INVALID_ARG = -1,     /* null pointer, bad size, non-finite input, bad option */
    BEM_ERR_MESH = -2,            /* open/non-manifold/inverted mesh, zero area, index out of range */
    BEM_ERR_OOM = -3,             /* device allocation failed or footprint over budget */
    BEM_ERR_DEVICE = -4,          /* a HIP call failed */
    BEM_ERR_UNSUPPORTED = -5      /* option not implemented */
} bem_status;

typedef struct { double re, im; } bem_complex;

typedef struct bem_problem bem_problem;   /* opaque; owned by the library until bem_destroy */

/* One penetrable domain Omega^j (paper eq. model).  Host arrays, copied by
 * bem_assemble.  Triangles are 0-based vertex triples ordered
 * counter-clockwise seen from the side the normal points to; the normal must
 * point out of the domain (paper: n^j points out of Omega^j).  A domain may
 * have several closed boundary components (e.g. a shell). */
typedef struct {
    const double *vertices;   int64_t n_vertices;    /* [n_vertices][3] */
    const int32_t *triangles; int64_t n_triangles;   /* [n_triangles][3] */
    bem_complex k;                                   /* k_j, Im k_j >= 0 */
    double rho;                                      /* rho_j > 0 */
} bem_domain;

/* operator storage modes */
#define BEM_OTF 0                  /* on-the-fly FP32 far field + FP64 sparse singular pass */
#define BEM_ASSEMBLED_FP32 1       /* dense complex64 matrix (FP32), applied by GEMV/GEMM */
#define BEM_ASSEMBLED_SPLIT_BF16 2 /* dense matrix plus BF16 hi/lo planes (3-term MFMA GEMM) */

/* flags */
#define BEM_DEVICE_PTRS 1u         /* vectors passed to apply/solve/rhs/evaluate are device pointers */
#define BEM_AUTOTUNE 2u            /* time candidate launch shapes of the pair kernel at set-up, of the
                                      single-layer pair kernel at its first use, and of the GEMM at first
                                      use per right-hand-side bucket; cache the pair and GEMM choices */

typedef struct {
    int mode;          /* BEM_OTF (default) or an assembled mode */
    int far_points;    /* must be 6 (the only far rule) */
    int ss_order;      /* Gauss-Legendre points per dimension of the singular rules (1..16), default 6 */
    int device;        /* HIP device ordinal */
    void *stream;      /* hipStream_t used for all work of this problem; NULL = default stream */
    uint32_t flags;    /* BEM_DEVICE_PTRS | BEM_AUTOTUNE */
} bem_assemble_opts;

/* Incident field kinds (paper eq. model: p_inc; numerical experiments). */
#define BEM_PLANE_WAVE 0     /* params [n_fields][5]: direction (3), amplitude re, im */
#define BEM_POINT_SOURCES 1  /* params [n_params][6]: position (3), amplitude re, im, field index */
#define BEM_PISTON_ARRAY 2   /* params [n_params][10]: centre (3), unit normal (3), radius, amp re, im, field index */

typedef struct {
    int kind;
    int32_t n_fields;       /* number of incident fields = number of right-hand sides */
    const double *params;   /* host array, layout per kind */
    int64_t n_params;       /* rows of params (plane waves: n_fields) */
} bem_incident;

/* OSRC block-diagonal preconditioner P (paper eqs. OSRC_prec, OSRC_prec_blocks,
 * OSRC_DtN_NtD_maps).  The paper solves the left-preconditioned system
 * P A u = P b, whose GMRES stops on the preconditioned residual.
 *   BEM_PRECOND_OSRC       plain forms: right preconditioning, GMRES on A P y = b,
 *                          u = P y (the preconditioned vectors are stored, as in
 *                          flexible GMRES); the Arnoldi residual, which stops it, is
 *                          the unpreconditioned weak-form residual ||b - A u||/||b||
 *   BEM_PRECOND_OSRC_LEFT  plain forms: the paper's left form, stopping on the
 *                          preconditioned residual ||P(b - A u)||/||P b||
 * The same P spectrum governs both (P A and A P are similar), so they take
 * about as many iterations; only the first stops at the stated tolerance of
 * the system itself. */
#define BEM_PRECOND_NONE 0
#define BEM_PRECOND_OSRC 1
#define BEM_PRECOND_OSRC_LEFT 2
/* Solver precision forms (compared at equal accuracy):
 *   BEM_PREC_FP32               plain GMRES on the FP32 operator (on-the-fly kernel, or the
 *                               dense FP32 matrix by GEMV with FP64 accumulation, one
 *                               right-hand side per launch)
 *   BEM_PREC_SPLIT_BF16_FGMRES  flexible GMRES: outer Arnoldi on the FP32 matrix with FP64
 *                               accumulation, inner block GMRES (to inner_tol) on the 3-term
 *                               split-BF16 MFMA GEMM, all right-hand sides in one launch
 *                               (problem assembled with BEM_ASSEMBLED_SPLIT_BF16)
 *   BEM_PREC_FP32_MFMA_FGMRES   the same with the FP32 MFMA GEMM as inner operator
 *                               (any assembled mode)
 *   BEM_PREC_HMATRIX            plain GMRES (or OSRC-preconditioned GMRES) on the
 *                               hierarchical matrix of bem_hmatrix_build (any mode);
 *                               the solution solves the compressed system
 *   BEM_PREC_HMATRIX_FGMRES     flexible GMRES: outer Arnoldi on the FP32 operator of the
 *                               problem's mode (on-the-fly kernel or dense GEMV) with its
 *                               FP64 residual, inner GMRES on the hierarchical matrix to
 *                               inner_tol (any mode)
 * With BEM_PRECOND_OSRC, plain GMRES runs on the right-preconditioned system
 * and stops on the unpreconditioned residual; with BEM_PRECOND_OSRC_LEFT on
 * the left-preconditioned one (stopping on the preconditioned residual).  The
 * flexible forms precondition their inner solves with either (inner GMRES on
 * P A z = P v) and keep stopping on the unpreconditioned FP64 residual.
 * Progress: with the environment variable BEM_PROGRESS=k (k > 0) the solvers
 * print one line to stderr every k Arnoldi steps. */
#define BEM_PREC_FP32 0
#define BEM_PREC_SPLIT_BF16_FGMRES 1
#define BEM_PREC_FP32_MFMA_FGMRES 2
#define BEM_PREC_HMATRIX 3          /* GMRES on the hierarchical matrix of bem_hmatrix_build */
#define BEM_PREC_HMATRIX_FGMRES 4   /* flexible GMRES, inner GMRES on the hierarchical matrix */

typedef struct {
    double tol;          /* relative residual target (paper: 1e-5) */
    int restart;         /* GMRES restart length (paper: 100) */
    int max_iter;        /* total iteration cap */
    int precond;         /* BEM_PRECOND_NONE, BEM_PRECOND_OSRC or BEM_PRECOND_OSRC_LEFT */
    int n_pade;          /* OSRC Pade terms */
    double r_eps;        /* OSRC damping length */
    double theta;        /* OSRC Pade branch-cut rotation */
    int precision;       /* BEM_PREC_FP32, BEM_PREC_SPLIT_BF16_FGMRES, BEM_PREC_FP32_MFMA_FGMRES,
                            BEM_PREC_HMATRIX or BEM_PREC_HMATRIX_FGMRES */
    double inner_tol;    /* inner tolerance of the flexible-GMRES refinement */
    int inner_restart;   /* inner GMRES restart length (0: 30) */
    int inner_max_iter;  /* inner iteration cap per outer step (0: 300) */
    double osrc_tol;     /* relative residual of the OSRC inner sparse solves (COCG).  0: inside
                            bem_solve one tenth of the tolerance of the GMRES it preconditions
                            (tol for the plain forms, inner_tol for the flexible forms' inner
                            solves), within [1e-10, 1e-4]; in bem_apply_preconditioner 1e-10.
                            A looser value makes each preconditioner apply cheaper and slightly
                            less exact; the solvers' stopping tests are unchanged */
} bem_solve_opts;

typedef struct {
    int32_t iterations;    /* (outer) GMRES iterations */
    int32_t converged;     /* the GMRES residual estimate reached tol: the unpreconditioned
                              residual, except with BEM_PRECOND_OSRC_LEFT (preconditioned) */
    double rel_residual;   /* true ||b - A u|| / ||b|| of the returned u (weak form, FP32 operator) */
} bem_solve_info;

/* Set up a problem: validate meshes, build geometry, quadrature points and the
 * FP64 singular correction on the device.  n_domains >= 1.  k0 with
 * Im k0 >= 0, rho0 > 0.  opts may be NULL (defaults).  On success *out owns
 * device memory until bem_destroy.  Errors: BEM_ERR_INVALID_ARG,
 * BEM_ERR_MESH, BEM_ERR_OOM, BEM_ERR_DEVICE. */
bem_status bem_assemble(const bem_domain *domains, int32_t n_domains, bem_complex k0, double rho0,
                        const bem_assemble_opts *opts, bem_problem **out);

/* y = A x for n_rhs vectors: the Galerkin PMCHWT matrix (weak form, no mass
 * matrix) applied to x.  x, y: [n_rhs][n_unknowns]; host or device memory per
 * BEM_DEVICE_PTRS; x and y must not overlap.  Runs on the problem's stream;
 * with device pointers the call returns after enqueueing the work. */
bem_status bem_apply(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs);

/* The single-layer operator alone (paper, Appendix A: V phi(x) = int G(x, y)
 * phi(y) ds_y, G = exp(i k0 |x - y|)/(4 pi |x - y|)), Galerkin P1 on the union
 * of all boundaries at the exterior wavenumber k0:
 *   y_i = sum_j <phi_i, V_k0 phi_j> x_j,
 * with the 6-point far rule on FP32 pairs plus the FP64 Sauter-Schwab
 * correction of touching pairs (the exterior V_k0 blocks of the PMCHWT matrix).
 * x, y: [n_rhs][total vertices], vertices in domain order (host or device per
 * BEM_DEVICE_PTRS).  The V-only correction is computed on the first call.
 * Available in every mode (it runs on the far-field pair path). */
bem_status bem_apply_single_layer(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs);

/* bem_apply without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operator, kernels and summation order as bem_apply, so the
 * result is bitwise the same.  Only for on-the-fly problems assembled with
 * BEM_DEVICE_PTRS: x and y are device arrays [n_rhs][n_unknowns] (not
 * overlapping), work is ordered on the problem's stream and the call returns
 * after enqueueing it.  The apply's scratch (trial records, pair-kernel partial
 * sums, point potentials: 16 (2 M + 3 T) + 80 (2 S + 1) M bytes, M = 6 T
 * quadrature points, T triangles, S the pair kernel's trial splits, each part
 * rounded up to 256 bytes) lives in a file-scope device array of
 * BEM_NOALLOC_SCRATCH_BYTES (256 MiB) that every GPU the library runs on holds
 * until the process ends; a problem needing more is rejected with
 * BEM_ERR_UNSUPPORTED (the 10,242-vertex sphere needs about 172 MB).  All
 * calls on one GPU share that array and it keeps the last call's contents
 * (the partial sums are cleared by a kernel on every call): calls that overlap
 * in time on one GPU (other streams or threads) race; calls on one stream are
 * ordered.  Errors: BEM_ERR_INVALID_ARG (null pointers, n_rhs < 0, assembled
 * mode, host vectors), BEM_ERR_UNSUPPORTED, BEM_ERR_DEVICE. */
#define BEM_NOALLOC_SCRATCH_BYTES (256ull << 20)
bem_status bem_apply_noalloc(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs);

/* bem_apply restricted to parts of the operator (parts: 1 = far field
 * (regular rule on every pair), 2 = singular correction; 3 = both). */
bem_status bem_apply_parts(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs, int parts);

/* bem_apply with an explicit kernel for assembled problems:
 *   BEM_APPLY_DEFAULT         as bem_apply (GEMV for one vector; for several, the GEMM of the
 *                             problem's mode: FP32 MFMA or split-BF16 MFMA)
 *   BEM_APPLY_GEMV            one GEMV per vector (FP32 matrix, FP64 accumulation)
 *   BEM_APPLY_MFMA_FP32       one FP32 MFMA GEMM for all vectors
 *   BEM_APPLY_MFMA_SPLIT_BF16 one 3-term split-BF16 MFMA GEMM for all vectors (problem
 *                             assembled with BEM_ASSEMBLED_SPLIT_BF16), tile shape and K
 *                             slices from the autotuner (BEM_AUTOTUNE) or the heuristic
 *   BEM_APPLY_MFMA_SPLIT_BF16_W4  the same GEMM forced to its 256 x 128 four-wave tile
 *   BEM_APPLY_MFMA_SPLIT_BF16_W8  the same GEMM forced to its 384 x 128 eight-wave tile
 *                             (both with heuristic K slices; for tests and measurements)
 * On-the-fly problems accept BEM_APPLY_DEFAULT and BEM_APPLY_HMATRIX. */
#define BEM_APPLY_DEFAULT 0
#define BEM_APPLY_GEMV 1
#define BEM_APPLY_MFMA_FP32 2
#define BEM_APPLY_MFMA_SPLIT_BF16 3
#define BEM_APPLY_MFMA_SPLIT_BF16_W4 4
#define BEM_APPLY_MFMA_SPLIT_BF16_W8 5
#define BEM_APPLY_HMATRIX 6   /* the hierarchical matrix of bem_hmatrix_build (any mode) */
bem_status bem_apply_with(bem_problem *p, const bem_complex *x, bem_complex *y, int32_t n_rhs, int kernel);

/* Right-hand side b_j = <gamma^{j,+} p_inc, phi> (eq. Galerkin_disc_rhs1) for
 * each incident field: b [n_fields][n_unknowns]. */
bem_status bem_rhs(bem_problem *p, const bem_incident *inc, bem_complex *b);

/* Solve A u = b for every incident field with GMRES (FP64 Arnoldi, zero
 * initial guess).  u: [n_fields][n_unknowns]; info: [n_fields] (host).
 * Returns BEM_WARN_NOT_CONVERGED when some field hit max_iter. */
bem_status bem_solve(bem_problem *p, const bem_incident *inc, const bem_solve_opts *opts,
                     bem_complex *u, bem_solve_info *info);

/* Solve A u = b for given right-hand sides b [n_rhs][n_unknowns]. */
bem_status bem_solve_rhs(bem_problem *p, const bem_complex *b, int32_t n_rhs, const bem_solve_opts *opts,
                         bem_complex *u, bem_solve_info *info);

/* Out = P y for n_rhs residual vectors y [n_rhs][n_unknowns], P the OSRC
 * block-diagonal preconditioner of opts (precond = either OSRC form, n_pade,
 * r_eps, theta; paper eqs. OSRC_prec, OSRC_prec_blocks, OSRC_DtN_NtD_maps):
 * per domain, Lambda_DtN M^-1 applied to the Dirichlet-equation rows and
 * Lambda_NtD M^-1 to the Neumann-equation rows, k = k0, with the paper's
 * permutation of the unknowns to [u_N; u_D] folded in: the Lambda_DtN result
 * is returned in the u_N positions and the Lambda_NtD result in the u_D
 * positions (GMRES on P A u = P b).  Inner sparse solves by COCG in FP64 to
 * the relative residual opts->osrc_tol, or 1e-10 when it is 0.  The call
 * returns once out is complete, with host or device pointers.  The problem
 * keeps the preconditioner's sparse-solve workspace (up to 2 GB) for the next
 * call with the same n_pade, r_eps, theta, osrc_tol and n_rhs; it is rebuilt
 * when they change and freed by bem_destroy. */
bem_status bem_apply_preconditioner(bem_problem *p, const bem_solve_opts *opts, const bem_complex *y,
                                    bem_complex *out, int32_t n_rhs);

/* Total pressure at points from traces u (paper eq. rep_formula_gen):
 * exterior p = p_inc + sum_j [DL_k0 u_D^j - SL_k0 u_N^j]; inside domain j
 * p = SL_kj((rho_j/rho_0) u_N^j) - DL_kj u_D^j.  points [n_points][3] (host
 * or device per flag); field [n_fields][n_points]; region [n_points]
 * (0 exterior, j >= 1 domain j from the solid-angle winding number, -1 for
 * points closer than 2 h_j to the boundary of some domain j, h_j the mean edge
 * length of its mesh: the 6-point rule is not accurate there; their field is
 * still computed, in the region the winding number gives).  inc may be NULL
 * (no incident term). */
bem_status bem_evaluate_field(bem_problem *p, const bem_complex *u, const bem_incident *inc,
                              const double *points, int64_t n_points,
                              bem_complex *field, int32_t *region);

/* Hierarchical-matrix compression of the PMCHWT matrix, the paper's device
 * for going beyond dense storage (its numerical experiments use H-matrices
 * with adaptive cross approximation).  The vertices of all boundaries are
 * clustered by recursive median bisection down to leaf_vertices per cluster; a
 * pair of clusters with max(diam) <= eta dist (bounding boxes of the supports
 * of the clusters' basis functions; see bem_hmatrix_plan) becomes a
 * low-rank block, built by adaptive cross approximation with partial pivoting
 * to the relative tolerance eps of its Frobenius norm (the entries of each
 * pivot row and column computed on demand, the stopping test confirmed on
 * sampled rows; kept dense when the rank would not halve its storage); pairs
 * of leaves are dense blocks with the FP64 singular correction.  Clusters
 * never mix boundaries (the tree splits between boundaries first).  Entries
 * are those of the assembled matrix (FP32 pairs, complex64 storage).  The
 * environment variable BEM_HMATRIX_ACA=complete selects complete pivoting on
 * fully computed blocks instead (to the tolerance eps of the largest entry),
 * for comparisons.  Replaces any previous hierarchical matrix of p; it is
 * applied by bem_apply_with(BEM_APPLY_HMATRIX) and used by solves with
 * precision BEM_PREC_HMATRIX.  eps in (0, 0.1], leaf_vertices in [8, 4096],
 * eta > 0.  info may be NULL. */
typedef struct {
    int64_t n_blocks, n_lowrank, n_dense;
    int64_t n_admissible;   /* blocks the tree made admissible (low rank, or dense when not compressible) */
    int64_t bytes;          /* storage of all blocks */
    int64_t dense_bytes;    /* the dense complex64 matrix, for comparison */
    int32_t max_rank;
    int32_t pad;
    double build_s;
} bem_hmatrix_info;
bem_status bem_hmatrix_build(bem_problem *p, double eps, int32_t leaf_vertices, double eta, bem_hmatrix_info *info);

/* The cluster and block trees bem_hmatrix_build would use for these domains,
 * computed on the host alone (no device needed).  A cluster's box bounds the
 * supports of its vertices' P1 functions (all triangles at each vertex), so
 * two vertices whose functions meet on touching triangles (the pairs that
 * get the Sauter-Schwab rules) lie in clusters at distance 0, which are never
 * admissible.  out4 (host, 4 values): [0] blocks, [1] admissible blocks,
 * [2] vertex pairs of the singular pattern (touching triangles within one
 * boundary), [3] of those, the pairs that fall in an admissible block (0 by
 * construction; bem_hmatrix_build fails with BEM_ERR_DEVICE otherwise).
 * Errors: BEM_ERR_INVALID_ARG (null pointers, leaf_vertices outside
 * [8, 4096], eta <= 0), BEM_ERR_MESH as in bem_assemble. */
bem_status bem_hmatrix_plan(const bem_domain *domains, int32_t n_domains, int32_t leaf_vertices, double eta,
                            int64_t *out4);

/* Continuous batching of solves (serving).  Requests are solved side by side,
 * each by its own host thread on its own stream (right-hand sides, Krylov
 * vectors, preconditioner and results stay on that stream).  A problem
 * attached to a batch hands every operator apply of its solves (bem_solve,
 * bem_solve_rhs) to the batch's dispatcher thread, which gathers the applies
 * submitted by the requests in flight (until every attached problem inside a
 * solve has submitted one, or for at most a window, 0.3 ms by default) and
 * launches them together
 * on the batch's own stream: the pair kernels of all on-the-fly problems of
 * one kernel variant as one grouped launch over their concatenated work lists
 * (up to 16 problems), then each problem's gathers, reductions, projections,
 * GEMVs, GEMMs or hierarchical-matrix products back to back.  Each problem's
 * work items, launch shapes and summation orders are its own, so a result is
 * bitwise the same whatever the mix.  Events order the batch's stream after
 * the request's input and the request's stream after the result.
 * bem_batch_create: a batch on `device` (its stream has the default priority).
 * bem_batch_attach: route p's solves through b (NULL: launch them directly
 * again); p and b on the same device; not while p is inside a solve.
 * bem_batch_set_window: the longest the dispatcher waits for the other
 * requests in a solve once one apply is pending (default 0.3 ms; 0 launches
 * at once; a long window makes the steps of all requests in a solve go in
 * lockstep, every dispatch holding one apply of each), 0 <= seconds <= 10.
 * bem_batch_stats: out6 = {dispatches, applies, grouped pair launches, of
 * them with several problems, most problems in one launch, pair work items}.
 * bem_batch_destroy: stops the dispatcher; destroy or detach every attached
 * problem first.  Errors: BEM_ERR_INVALID_ARG, BEM_ERR_DEVICE. */
typedef struct bem_batch bem_batch;
bem_status bem_batch_create(int device, bem_batch **out);
bem_status bem_batch_attach(bem_problem *p, bem_batch *b);
bem_status bem_batch_set_window(bem_batch *b, double seconds);
bem_status bem_batch_stats(bem_batch *b, int64_t *out6);
void bem_batch_destroy(bem_batch *b);

int64_t bem_num_unknowns(const bem_problem *p);

/* Device bytes a problem would hold (admission control). */
bem_status bem_footprint_bytes(const bem_domain *domains, int32_t n_domains, const bem_assemble_opts *opts,
                               int32_t n_rhs, int32_t restart, uint64_t *bytes);

/* Launch shape chosen for the pair kernel: test points per lane and trial
 * splits (out[0], out[1]). */
bem_status bem_pair_launch_shape(const bem_problem *p, int32_t *out2);

/* Kernel timing of the last bem_apply on this problem, in milliseconds,
 * measured with HIP events on the problem's stream: [0] whole apply,
 * [1] far-field pair kernel, [2] singular sparse pass + scatter, [3] gather. */
bem_status bem_last_timings(const bem_problem *p, double *ms4);

void bem_destroy(bem_problem *p);

/* Message of the last non-OK status returned on this thread. */
const char *bem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BEM_MI355X_H */
