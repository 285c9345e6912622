/*
 * mgl.h -- C ABI of the learnable graph-convolution multigrid V-cycle for
 * AMD Instinct MI355X (gfx950).
 *
 * The library solves A u = f with the stationary iteration
 *     u^m = u^{m-1} + B_Theta (f - A u^{m-1})                 (paper Sec. 1)
 * whose approximate inverse B_Theta is one learnable V-cycle (paper Alg. 2):
 * on every level l < J-1 (0 = finest) the smoother is
 *     delta = theta_l D_A^{-1} (f - A_l u),   u <- u + eta_l Phi_B,l(delta)
 * (Sec. 3, learnable smoother; damped Jacobi B_l = D_A^{-1}, Sec. 2.3), the
 * restriction is r_c = R_l Phi_R,l(f - A_l u) and the prolongation adds
 * Phi_P,l(P_l e_c) (Sec. 3, learnable transfers), and level J-1 is solved
 * exactly.  Every graph convolution is a polynomial in the neighbour-mean
 * operator M_l = D_g^{-1} A_g of the level's graph (Sec. 3.3 eq. graph-conv-
 * matrix; K = 1 is SAGEConv with mean aggregation, Sec. 3.2; order K per the
 * polynomial-smoother remark of Sec. 3.3):
 *     Phi(x) = sum_{k=0..K} c_k M^k x .
 * The graph of level l is {(i, j): A_ij != 0, i != j} unless given (Sec. 2.1).
 * mg_params selects the aggregation operator G in place of M (weighted or
 * symmetric normalisation) and a Chebyshev basis for the coefficients.
 *
 * Conventions for every entry point:
 *  - Return an mg_status; they never abort and never throw.  On failure a
 *    thread-local message is available from mg_last_error().
 *  - Vectors are device arrays of n x B values, row-major with the B
 *    right-hand sides contiguous (element (i, b) at i*B + b).  Their element
 *    type depends on the context precision: double for MG_FP64, float for
 *    MG_FP32 and MG_FP32_BF16 ("cycle type").  Solver-level vectors
 *    (mg_solve, mg_residual, mg_refine_step*) are always double.
 *  - Work is enqueued on the HIP stream passed in (hipStream_t, may be NULL
 *    for the default stream) and is asynchronous unless stated otherwise.
 *  - Columns are independent: a column's result does not depend on the other
 *    columns, except parameter gradients, which sum over all columns.
 *  - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef MGL_H
#define MGL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx;

typedef enum {
    MG_OK = 0,
    MG_ERR_INVALID_ARG = 1,   /* null pointer, bad size or option */
    MG_ERR_SHAPE = 2,         /* inconsistent matrix shapes or malformed CSR */
    MG_ERR_OOM = 3,           /* device allocation failed or workspace too small */
    MG_ERR_HIP = 4,           /* a HIP call or kernel launch failed */
    MG_ERR_NOT_CONVERGED = 5, /* mg_solve: some column missed rtol in max_outer cycles */
    MG_ERR_DIVERGED = 6,      /* mg_solve: some column's residual became non-finite or grew */
    MG_ERR_STATE = 7,         /* call not valid in this context state */
    MG_ERR_UNSUPPORTED = 8    /* feature not available for these inputs */
} mg_status;

typedef enum {
    MG_FP64 = 0,       /* cycle in FP64 */
    MG_FP32 = 1,       /* cycle in FP32, FP64 outer residual / update / coarsest solve */
    MG_FP32_BF16 = 2   /* as MG_FP32, with the smoother and transfer intermediates stored in BF16 */
} mg_precision;

/* Host CSR matrix, 0-based, column indices sorted and unique within a row.
 * The library copies what it needs during mg_setup; the arrays may be freed
 * afterwards. */
typedef struct {
    int32_t nrows, ncols;
    int64_t nnz;
    const int32_t* rowptr;   /* [nrows + 1] */
    const int32_t* col;      /* [nnz] */
    const double* val;       /* [nnz]; ignored for graph patterns */
} mg_csr;

/* Multigrid hierarchy (paper Sec. 2.2).  Level 0 is the finest. */
typedef struct {
    int32_t nlevels;         /* J >= 2 */
    const mg_csr* A;         /* [J] system matrices A_l, nonzero diagonal */
    const mg_csr* P;         /* [J-1] prolongations, n_l x n_{l+1} */
    const mg_csr* R;         /* [J-1] restrictions n_{l+1} x n_l, or NULL for R_l = P_l^T */
    const mg_csr* G;         /* [J] graph patterns (diagonal ignored), or NULL for the
                                off-diagonal nonzero pattern of A_l */
    int32_t ncolumn_values;  /* 0: every column solves with A_l's values.  nrhs: column b solves
                                its own operators A_l^(b) on the pattern of A_l (a batch of
                                requests of one grid: per-request values, shared pattern, graph,
                                P and R; A_l's own values are then not read).  Every column's
                                off-diagonal values on the pattern and its diagonal must be
                                nonzero, so the graph (A_l's off-diagonal pattern) is the same as
                                each column's own.  Mean aggregation only; no reverse sweep and no
                                FGMRES in such a context (MG_ERR_UNSUPPORTED) */
    const double* const* column_values;  /* [J * nrhs] when ncolumn_values > 0:
                                column_values[l * nrhs + b] points at the nnz(A_l) values of
                                A_l^(b) in the CSR order of A_l's pattern (may repeat pointers) */
} mg_hierarchy;

/* Learnable parameters Theta (paper Sec. 3, parameter set).  values is a host
 * array of mg_num_params(J, KB, KR, KP) doubles laid out per level
 * l = 0 .. J-2 as
 *     [theta_l, eta_l, cB_l[0..KB], cR_l[0..KR], cP_l[0..KP]] .
 * Identity initialisation (Sec. 3.4): theta = omega, eta = 1, c_0 = 1,
 * c_k = 0 for k > 0, which is the classical V-cycle (Alg. 1), in either basis
 * (T_0 = 1).  The library evaluates every convolution as a polynomial in G by
 * Horner's rule; Chebyshev coefficients are converted to power-series
 * coefficients once (at setup and in mg_set_params), and parameter gradients
 * are returned with respect to the coefficients in the chosen basis. */
typedef enum {
    MG_BASIS_MONOMIAL = 0,   /* Phi(x) = sum_k c_k G^k x (SAGEConv for K = 1) */
    MG_BASIS_CHEBYSHEV = 1   /* Phi(x) = sum_k c_k T_k(-G) x: the ChebConv layer (Sec. 3.2) with the
                                rescaled Laplacian 2 (I - G) / lambda_max - I, lambda_max = 2 */
} mg_basis;

typedef enum {
    MG_AGG_MEAN = 0,         /* G = D_g^{-1} A_g, the neighbour mean (Sec. 3.2) */
    MG_AGG_WEIGHTED = 1,     /* G = D_w^{-1} W, W_ij = |A_ij| on the graph of A (|G_ij| for a given
                                graph, which then needs values); D_w = diag(sum_j W_ij): edge
                                weights from matrix entries (Sec. 2.1) */
    MG_AGG_SYM = 2           /* G = D_g^{-1/2} A_g D_g^{-1/2}, the symmetric normalisation of ChebConv */
} mg_aggregation;

typedef struct {
    int32_t KB, KR, KP;      /* orders of Phi_B, Phi_R, Phi_P (0..8) */
    int32_t nu_pre, nu_post; /* smoothing steps per level (0..8) */
    const double* values;
    int32_t basis;           /* mg_basis of the coefficients c in values */
    int32_t aggregation;     /* mg_aggregation: the graph operator G the convolutions use */
} mg_params;

enum {
    MG_FLAG_BACKWARD = 1,   /* reserve buffers for mg_*_backward */
    MG_FLAG_NO_TAIL = 2,    /* never run the coarse levels as one LDS-resident kernel */
    MG_FLAG_NO_TILES = 4,   /* never run a K-hop convolution as one fused LDS-tile kernel */
    MG_FLAG_NO_COMPACT = 8  /* mg_solve: keep cycling all nrhs columns (by default, at its periodic
                               checks the solver narrows the cycle to the columns still iterating,
                               rounded up to 16; a column's arithmetic and result do not change) */
};

typedef struct {
    int32_t precision;       /* mg_precision */
    int32_t nrhs;            /* B, 1..256 */
    int32_t max_outer;       /* mg_solve: cycle cap (>= 1) */
    int32_t check_every;     /* mg_solve: host reads the active-column count every this many cycles */
    double rtol;             /* mg_solve: stop a column when ||f - A u|| <= rtol ||f|| */
    double diverge_factor;   /* mg_solve: a column diverges when its residual norm exceeds
                                this factor times the initial one or is not finite; <= 0 disables */
    int32_t flags;           /* MG_FLAG_* */
} mg_options;

typedef struct {
    int32_t iters;           /* cycles applied to the column */
    int32_t status;          /* MG_OK, MG_ERR_NOT_CONVERGED or MG_ERR_DIVERGED */
    double relres;           /* final ||f - A u||_2 / ||f||_2 (FP64); 0 when f = 0 */
} mg_rhs_info;

/* Number of doubles in the parameter vector. */
int64_t mg_num_params(int32_t nlevels, int32_t KB, int32_t KR, int32_t KP);

/* Device bytes the context needs (workspace) and the size of one forward
 * checkpoint (ckpt) for the backward entry points.  No device work. */
mg_status mg_workspace_bytes(const mg_hierarchy* h, const mg_params* p, const mg_options* o,
                             size_t* workspace_bytes, size_t* ckpt_bytes);

/* Validate the hierarchy, build the device data structures (ELL matrices,
 * inverse diagonals and degrees, FP32 copies, the coarsest-level inverse by
 * Gauss-Jordan elimination with partial pivoting in FP64) and return a
 * context.  workspace: caller-owned device memory of at least the size
 * reported by mg_workspace_bytes (kept for the context's lifetime), or NULL
 * to let the library allocate it.  FP32/BF16 contexts with nrhs a multiple
 * of 16 also tile the levels of >= 2048 rows for the fused K-hop
 * convolution (unless MG_FLAG_NO_TILES); the tile lists (about 50 bytes per
 * unknown of those levels at K = 3) are allocated by the library outside
 * the workspace and freed by mg_destroy.  Synchronises `stream` before
 * returning. */
mg_status mg_setup(const mg_hierarchy* h, const mg_params* p, const mg_options* o,
                   void* workspace, size_t workspace_bytes, void* stream, mg_ctx** out);

/* Replace Theta (same layout and orders as at setup).  Synchronises `stream`. */
mg_status mg_set_params(mg_ctx* ctx, const double* values, void* stream);

/* Per-column operator contexts (mg_hierarchy.ncolumn_values = nrhs): replace
 * column b's operators A_l^(b) on every level, e.g. to start a new request in a
 * column slot that a finished one left (continuous batching of requests of
 * one grid).  values: host array [J] of pointers to nnz(A_l) doubles in the
 * CSR order of the pattern given at setup, with the same rules as at setup
 * (finite, nonzero on the pattern); the coarsest inverse is recomputed.  The
 * other columns are not touched.  Synchronises `stream`; must not overlap a
 * solve on the context.  MG_ERR_STATE for a context with shared operators,
 * MG_ERR_SHAPE (context unchanged) for values off the rules or a singular
 * coarsest operator.  The first call allocates a pinned host buffer for one
 * column's arrays of every level, kept by the context until mg_destroy. */
mg_status mg_load_column(mg_ctx* ctx, int32_t b, const double* const* values, void* stream);

/* Change mg_solve's options after setup (same meaning and limits as the
 * mg_options fields). */
mg_status mg_set_solver_options(mg_ctx* ctx, int32_t max_outer, int32_t check_every, double rtol,
                                double diverge_factor);

/* One learnable V-cycle on the finest level, in place:
 *     u <- LMG(A_0, f, u, Theta)                                 (Alg. 2)
 * f, u: cycle-type device vectors [n_0 x B].  ckpt: device buffer of
 * ckpt_bytes to record what mg_vcycle_backward needs, or NULL. */
mg_status mg_vcycle(mg_ctx* ctx, const void* f, void* u, void* ckpt, void* stream);

/* Reverse of the mg_vcycle call recorded in ckpt (Sec. 3.1, training by
 * back-propagation).  Given gu_out = dL/du_out, writes gu_in = dL/du_in and
 * gf = dL/df (cycle-type vectors, either may be NULL) and gparams = dL/dTheta
 * (device, mg_num_params doubles, overwritten; NULL to skip).  Requires
 * MG_FLAG_BACKWARD at setup, symmetric A_l and a symmetric graph. */
mg_status mg_vcycle_backward(mg_ctx* ctx, const void* ckpt, const void* gu_out,
                             void* gu_in, void* gf, double* gparams, void* stream);

/* FP64 outer residual r = f - A_0 u (r may be NULL) and its per-column
 * 2-norms (norms: device double [B], may be NULL). */
mg_status mg_residual(mg_ctx* ctx, const double* f, const double* u, double* r,
                      double* norms, void* stream);

/* Residual loss of training (paper Sec. 3.1, Alg. 3: the loss is the residual
 * of the linear system after the unrolled cycles) and its gradients, all in
 * FP64 on the device.  With r_b = f_b - A_0 u_b per column b:
 *   MG_LOSS_MEAN_REL_SQ: L = (1/B) sum_b ||r_b||^2 / ||f_b||^2  (a column with
 *       f_b = 0 contributes 0 and gets zero gradients)
 *       dL/du_b = -(2/B) A_0^T r_b / ||f_b||^2
 *       dL/df_b = (2/B) (r_b / ||f_b||^2 - ||r_b||^2 f_b / ||f_b||^4)
 *   MG_LOSS_RESID_NORM:  L = sum_b ||r_b||_2  (Alg. 3's residual norm, summed
 *       over the columns), dL/du_b = -A_0^T r_b / ||r_b||, dL/df_b = r_b / ||r_b||
 *       (zero for a column with r_b = 0).
 * f, u: device double [n_0 x B].  gseed: device double [1], a factor on both
 * gradients (the cotangent of L from the caller's graph), or NULL for 1.
 * loss: device double [1] or NULL.  gu, gf: device double [n_0 x B] or NULL;
 * they must not overlap f, u or each other.  gu needs a symmetric A_0 and a
 * context set up with MG_FLAG_BACKWARD (MG_ERR_UNSUPPORTED otherwise).
 * Overwrites the context's FP64 scratch vector (not f or u). */
typedef enum {
    MG_LOSS_MEAN_REL_SQ = 0,
    MG_LOSS_RESID_NORM = 1
} mg_loss_kind;
mg_status mg_residual_loss(mg_ctx* ctx, int32_t kind, const double* f, const double* u, const double* gseed,
                           double* loss, double* gu, double* gf, void* stream);

/* One outer iteration of the solver in refinement form:
 *     u_out = u_in + LMG_p(A_0, fl_p(f - A_0 u_in), 0)
 * with the residual and the update in FP64 and the cycle in the context
 * precision p.  f, u_in, u_out: device double [n_0 x B]; u_out may equal
 * u_in.  ckpt as for mg_vcycle. */
mg_status mg_refine_step(mg_ctx* ctx, const double* f, const double* u_in, double* u_out,
                         void* ckpt, void* stream);

/* Reverse of mg_refine_step: gu_in = gu_out - A_0^T C^T gu_out,
 * gf = C^T gu_out, where C is the cycle at zero initial guess.  Vectors are
 * device double; gu_in may equal gu_out; gf and gparams may be NULL. */
mg_status mg_refine_step_backward(mg_ctx* ctx, const void* ckpt, const double* gu_out,
                                  double* gu_in, double* gf, double* gparams, void* stream);

/* Solve A u = f for all B columns: refinement steps from the given u until
 * every column meets rtol (a column stops updating at the first iterate that
 * meets it), diverges, or max_outer cycles ran.  f, u: device double
 * [n_0 x B].  info: host array [B] (may be NULL).  Blocks the calling thread
 * (it reads the active count every check_every cycles).  Returns MG_OK,
 * MG_ERR_NOT_CONVERGED or MG_ERR_DIVERGED. */
mg_status mg_solve(mg_ctx* ctx, const double* f, double* u, mg_rhs_info* info, void* stream);

/* ---------------------------------------------------------------- Krylov and FMG
 * The trained cycle also serves as a preconditioner of flexible GMRES, either
 * as one V-cycle or inside full multigrid (paper Sec. 4.2, preconditioner
 * experiments, and its FMG paragraph). */

/* Full multigrid (nested iteration) with one learnable cycle per level:
 * f_0 = f, f_{l+1} = R_l Phi_R,l(f_l) (the cycle's own restriction);
 * u_{J-1} = A_{J-1}^{-1} f_{J-1}; for l = J-2 .. 0:
 * u_l = LMG(A_l, f_l, Phi_P,l(P_l u_{l+1})) (the cycle's own prolongation).
 * f, u: cycle-type device vectors [n_0 x B]; u is overwritten (its input
 * value is not used).  Uses the context's per-level buffers, like mg_vcycle. */
mg_status mg_fmg(mg_ctx* ctx, const void* f, void* u, void* stream);

typedef enum {
    MG_PC_NONE = 0,     /* z = fl_p(v): unpreconditioned (up to rounding to the cycle type) */
    MG_PC_VCYCLE = 1,   /* z = LMG_p(A_0, fl_p(v), 0): one learnable V-cycle */
    MG_PC_FMG = 2       /* z = FMG_p(fl_p(v)) */
} mg_preconditioner;

typedef struct {
    int32_t restart;    /* m: basis vectors per restart cycle, 1..63 */
    int32_t max_iter;   /* cap on a column's FGMRES iterations (preconditioner calls), >= 1 */
    double rtol;        /* stop a column when ||f - A u|| <= rtol ||f|| */
    int32_t precond;    /* mg_preconditioner */
    double reorth;      /* second Gram-Schmidt pass for a vector when, in some active column,
                           ||w after the first pass|| < reorth * ||w||.  The first pass leaves
                           the new vector orthogonal to about eps / reorth, so 0.1 keeps the
                           basis orthogonal to about ten units of roundoff per vector and
                           0.70710678 ("twice is enough") to working precision; 0 never
                           reorthogonalises (classical Gram-Schmidt), >= 1 always does */
} mg_krylov_options;

/* Device bytes of the Krylov workspace for these options: (m+1) FP64 basis
 * vectors, m preconditioned vectors in the cycle type, one FP64 vector and
 * O(m^2 B) per-column scalars.  No device work. */
mg_status mg_fgmres_workspace_bytes(const mg_ctx* ctx, const mg_krylov_options* o, size_t* bytes);

/* Solve A_0 u = f by restarted flexible GMRES with right preconditioning
 * (Saad 1993) per column, from the given u.  The preconditioner runs in the
 * context precision; A z, the orthonormal basis (classical Gram-Schmidt with a
 * second pass as o->reorth selects), the Hessenberg least-squares problem and
 * the iterate are FP64.  Each restart begins with the true FP64 residual; a column stops at
 * the first iteration whose least-squares residual estimate meets rtol (or
 * when its Krylov space becomes invariant) and is finished when its true
 * residual does.  info[b].iters counts the column's iterations.  f, u: device
 * double [n_0 x B].  work: caller device memory of mg_fgmres_workspace_bytes,
 * or NULL: the library then allocates it on the first call and keeps it
 * (growing it when a larger restart needs more) until mg_destroy.  Blocks the
 * calling thread (reads the active-column count every iteration).  Returns
 * MG_OK, MG_ERR_NOT_CONVERGED (a column missed rtol in max_iter iterations)
 * or MG_ERR_DIVERGED (a column's residual is not finite). */
mg_status mg_fgmres(mg_ctx* ctx, const double* f, double* u, const mg_krylov_options* o,
                    void* work, size_t work_bytes, mg_rhs_info* info, void* stream);

/* Allocation-free form of mg_fgmres, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as mg_fgmres without the
 * workspace: the Krylov workspace is a static buffer of
 * MG_FGMRES_STATIC_MAX_BYTES inside the library, one per GPU, held until the
 * process ends; the call allocates no device or host memory.  Returns
 * MG_ERR_OOM, before any device work, when mg_fgmres_workspace_bytes for these
 * options exceeds that size (e.g. 129 x 129 unknowns with 16 columns fit a
 * restart of 30; the 513 x 513 workload with 64 columns does not fit any).
 * No part of the buffer needs to start at zero (each solve initialises what
 * it reads), and it keeps the last call's contents.  Every call on one GPU
 * shares the buffer: calls that overlap on one GPU, from any context or
 * stream, race and must be serialised by the caller. */
#define MG_FGMRES_STATIC_MAX_BYTES (64u << 20)
mg_status mg_fgmres_static(mg_ctx* ctx, const double* f, double* u, const mg_krylov_options* o,
                           mg_rhs_info* info, void* stream);

/* Per-level sizes: n_l for l < J (out: host int64 [J]) plus ELL widths of
 * A_l (wA: host int32 [J], may be NULL). */
mg_status mg_level_info(const mg_ctx* ctx, int64_t* n, int32_t* wA);

/* Instrumentation.  Kernel families for mg_timing_start. */
enum {
    MG_KF_NONE = 0,
    MG_KF_HOP = 1,       /* graph-convolution hops (neighbour mean + axpy) */
    MG_KF_RESID = 2,     /* residual / Jacobi-scaled residual sweeps */
    MG_KF_RESTRICT = 3,  /* restriction (with fused residual or last hop) */
    MG_KF_PROLONG = 4,   /* prolongation (with fused correction) */
    MG_KF_OUTER = 5,     /* FP64 outer residual with column norms */
    MG_KF_KRYLOV = 6,    /* FGMRES Gram-Schmidt sweeps (dot products, basis updates) */
    MG_KF_CONV = 7       /* fused K-hop graph convolutions over LDS tiles */
};

/* Start timing every launch of one kernel family on one level (level -1:
 * every level; the FP64 outer residual counts as level 0): a HIP event pair
 * is recorded around each such launch on its stream, and the algorithmic
 * bytes of the launch (each operand streamed once: vectors read and
 * written, ELL indices and values, per-row scalars) are added up.
 * kernel_family MG_KF_NONE stops timing.  Clears earlier records. */
mg_status mg_timing_start(mg_ctx* ctx, int32_t kernel_family, int32_t level);

/* Number of timed launches, their summed duration (milliseconds, from the
 * event pairs) and their summed algorithmic bytes.  Synchronises on the
 * recorded events. */
mg_status mg_timing_read(mg_ctx* ctx, int64_t* launches, double* total_ms, double* total_bytes);

/* ---------------------------------------------------------------- setup helpers
 * Host-side builder of structured hierarchies (per-request setup when
 * serving; the hierarchy is input data of the V-cycle).
 * -div(a grad u) = f on the unit square, P1 elements on the uniform mesh of
 * `side` points per direction (side = 2^k + 1) with every cell split along
 * its south-west/north-east diagonal, homogeneous Dirichlet boundary
 * eliminated, a piecewise constant on an nb x nb array of square blocks
 * (blocks[bj * nb + bi] > 0 covers [bi/nb, (bi+1)/nb) x [bj/nb, (bj+1)/nb)),
 * P = nested linear interpolation, R = P^T and Galerkin coarse operators
 * A_{l+1} = P^T A_l P (paper Sec. 2.2) symmetrised with off-diagonal
 * round-off residue (|a_ij| <= 1e-11 sqrt(|a_ii a_jj|)) removed; coarsening
 * stops at a coarsest x coarsest interior.  Returns MG_ERR_SHAPE when side
 * does not coarsen to that size.  The object owns its arrays. */
typedef struct mg_host_hierarchy mg_host_hierarchy;
mg_status mg_square_hierarchy(int32_t side, int32_t nb, const double* blocks, int32_t coarsest,
                              mg_host_hierarchy** out);
/* Fill `view` with pointers into `h` (valid until mg_host_hierarchy_free). */
mg_status mg_host_hierarchy_view(const mg_host_hierarchy* h, mg_hierarchy* view);
void mg_host_hierarchy_free(mg_host_hierarchy* h);

/* Release the context (and the workspace if the library allocated it).
 * Waits for the context's work to finish.  NULL is ignored. */
void mg_destroy(mg_ctx* ctx);

/* Message describing the last failure on this thread ("" if none). */
const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGL_H */
