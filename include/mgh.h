/*
 * mgh.h -- C ABI of the learnable V-cycle for complex Helmholtz systems with
 * two features per node, for AMD Instinct MI355X (gfx950).
 *
 * Model problem (paper Sec. 4.2, Helmholtz subsection): -Lap u - k^2 u = f
 * with an impedance boundary, discretised as a complex symmetric A u = f.
 * A complex value is carried as d = 2 node features (real part, imaginary
 * part), and every graph convolution mixes them with 2 x 2 real weight
 * matrices:
 *     Phi(x)_i = sum_{k=0..K} W_k (M^k x)_i ,   M = D_g^{-1} A_g
 * (the neighbour mean on the graph of A_l acting on nodes, W_k acting on the
 * two features of a node).  K = 1 is SAGEConv with mean aggregation, whose
 * self weight is W_0 here and whose neighbour weight is W_1 (Sec. 3.2); the
 * higher orders follow the polynomial remark of Sec. 3.3.
 * Per level the smoother is either
 *   Jacobi:  delta = theta_l D_A^{-1} (f - A_l u),  u <- u + eta_l Phi_B,l(delta)
 *            (D_A the complex diagonal; Sec. 3, learnable smoother), or
 *   GMRES:   r = f - A_l u,  delta_0 = theta_l Phi_B,l(r),
 *            u <- u + eta_l GMRES(A_l, r, delta_0, v)
 *            (v steps of GMRES from delta_0, complex arithmetic; Sec. 3, the
 *            Krylov-smoother form),
 * the restriction is r_c = R_l Phi_R(r) and the prolongation adds
 * Phi_P(P_l e_c), with Phi_R and Phi_P shared by all levels (Sec. 4.2), and
 * the coarsest level is solved exactly.  With GMRES levels the cycle is not
 * affine in its input; it is used as an iteration u <- LMG(A, f, u), or as a
 * (flexible) preconditioner of FGMRES, alone or inside full multigrid.
 *
 * Conventions: status codes, mg_csr and the Krylov options are those of
 * mgl.h.  Complex vectors are device arrays of n x B complex values,
 * row-major with the B right-hand sides contiguous and every complex value
 * stored as (real, imaginary): element (i, b) at 2 (i B + b) and
 * 2 (i B + b) + 1 (the memory layout of a C99 or std::complex array [n][B]).
 * Cycle-type vectors hold double for MG_FP64 and float for MG_FP32 contexts;
 * solver-level vectors (mgh_residual, mgh_fgmres) are always double.  Work is
 * enqueued on the HIP stream passed in (may be NULL) and is asynchronous
 * unless stated otherwise.  Columns are independent.  A context is not
 * thread-safe.  Errors: mgh_last_error() describes the last failure on the
 * calling thread.
 */
#ifndef MGH_H
#define MGH_H

#include "mgl.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgh_ctx mgh_ctx;

/* Host complex CSR matrix, 0-based, column indices sorted and unique within
 * a row.  Copied during mgh_setup. */
typedef struct {
    int32_t nrows, ncols;
    int64_t nnz;
    const int32_t* rowptr;   /* [nrows + 1] */
    const int32_t* col;      /* [nnz] */
    const double* re;        /* [nnz] real parts */
    const double* im;        /* [nnz] imaginary parts */
} mgh_ccsr;

/* Hierarchy, level 0 the finest.  A_l complex with nonzero diagonal; P_l real
 * (n_l x n_{l+1}); R_l = P_l^T when R is NULL.  The graph of level l is the
 * off-diagonal nonzero pattern of A_l (Sec. 2.1). */
typedef struct {
    int32_t nlevels;         /* J >= 2 */
    const mgh_ccsr* A;       /* [J] */
    const mg_csr* P;         /* [J-1] */
    const mg_csr* R;         /* [J-1] or NULL */
} mgh_hierarchy;

typedef enum { MGH_JACOBI = 0, MGH_GMRES = 1 } mgh_smoother;

/* Parameters.  values: host array of mgh_num_params(J, KB, KR, KP) doubles,
 * per level l = 0 .. J-2
 *     [theta_l, eta_l, W_B,l[0] .. W_B,l[KB]]
 * (each W a 2 x 2 matrix, row-major: W[0][0], W[0][1], W[1][0], W[1][1];
 * feature 0 is the real part), followed by the shared W_R[0..KR] and
 * W_P[0..KP].  Identity initialisation: W_0 = I, W_k = 0 for k > 0, eta = 1,
 * theta = omega on Jacobi levels and 0 on GMRES levels (the classical
 * smoothers). */
typedef struct {
    int32_t KB, KR, KP;          /* convolution orders, 0..8 */
    const int32_t* smoother;     /* [J-1] mgh_smoother of each level */
    const int32_t* nu_pre;       /* [J-1] pre-smoothing steps, 0..8 */
    const int32_t* nu_post;      /* [J-1] post-smoothing steps, 0..8 */
    int32_t gmres_steps;         /* v of every GMRES smoothing step, 1..8 */
    const double* values;
} mgh_params;

typedef struct {
    int32_t precision;           /* MG_FP64 or MG_FP32 (cycle type) */
    int32_t nrhs;                /* B, 1..256 */
} mgh_options;

int64_t mgh_num_params(int32_t nlevels, int32_t KB, int32_t KR, int32_t KP);

/* Validate the hierarchy and build the device data (ELL matrices, complex
 * inverse diagonals, neighbour lists and inverse degrees, the coarsest-level
 * inverse by complex Gauss-Jordan elimination with partial pivoting in FP64,
 * per-level buffers).  The library allocates and owns all device memory of
 * the context.  Synchronises `stream` before returning. */
mg_status mgh_setup(const mgh_hierarchy* h, const mgh_params* p, const mgh_options* o, void* stream,
                    mgh_ctx** out);

/* Replace the parameter values (same orders and smoother plan). */
mg_status mgh_set_params(mgh_ctx* ctx, const double* values, void* stream);

/* One learnable V-cycle on the finest level, in place: u <- LMG(A_0, f, u)
 * (Alg. 2 with the per-level smoothers above).  f, u: cycle-type complex
 * vectors [n_0 x B]; f and u must not overlap (MG_ERR_INVALID_ARG). */
mg_status mgh_vcycle(mgh_ctx* ctx, const void* f, void* u, void* stream);

/* Full multigrid with one cycle per level (Sec. 4.2, FMG paragraph):
 * f_{l+1} = R_l Phi_R(f_l), exact coarsest solve, u_l = LMG(A_l, f_l,
 * Phi_P(P_l u_{l+1})).  f, u: cycle-type complex vectors that must not
 * overlap; u is overwritten. */
mg_status mgh_fmg(mgh_ctx* ctx, const void* f, void* u, void* stream);

/* FP64 residual r = f - A_0 u (r may be NULL) and its per-column 2-norms
 * (norms: device double [B], may be NULL).  f, u, r: double complex. */
mg_status mgh_residual(mgh_ctx* ctx, const double* f, const double* u, double* r, double* norms,
                       void* stream);

/* Complex flexible GMRES(restart) per column with right preconditioning
 * (Saad 1993) from the given u: the preconditioner (none, one cycle from
 * zero, or FMG) runs in the context precision on fl(v); A z, the orthonormal
 * basis (classical Gram-Schmidt with a second pass as o->reorth selects,
 * Hermitian inner products), the Hessenberg least-squares problem (complex
 * Givens rotations) and the iterate are FP64.  A restart begins with the true
 * residual; a column stops iterating when its residual estimate meets rtol
 * and is finished when its true residual does.  f, u: double complex
 * [n_0 x B].  The Krylov workspace ((restart + 1) FP64 basis vectors,
 * restart cycle-type vectors) is allocated by the library on first use and
 * kept until mgh_destroy.  info: host [B] or NULL.  Blocks the calling thread
 * (reads the active-column count every iteration).  Returns MG_OK,
 * MG_ERR_NOT_CONVERGED or MG_ERR_DIVERGED. */
mg_status mgh_fgmres(mgh_ctx* ctx, const double* f, double* u, const mg_krylov_options* o,
                     mg_rhs_info* info, void* stream);

/* Stationary iteration u <- LMG(A_0, f, u) per column from the given u
 * (the paper's use of the cycle as an iterative solver, Sec. 4.2 tables):
 * a column stops at the first iterate with ||f - A_0 u|| <= rtol ||f||
 * (FP64 residual after every cycle, decided on the device) and then keeps
 * that iterate, or when its residual is not finite; at most max_cycles
 * cycles.  Needs an MG_FP64 context (MG_ERR_UNSUPPORTED otherwise: the cycle
 * is not affine, so lower-precision cycles have no refinement form).  f, u:
 * double complex [n_0 x B], not overlapping.  Blocks the calling thread (reads
 * the active-column count every check_every cycles).  info: host [B] or NULL;
 * info[b].iters counts the cycles applied to column b.  Returns MG_OK,
 * MG_ERR_NOT_CONVERGED or MG_ERR_DIVERGED. */
mg_status mgh_solve(mgh_ctx* ctx, const double* f, double* u, double rtol, int32_t max_cycles,
                    int32_t check_every, mg_rhs_info* info, void* stream);

/* Level sizes n_l (host int64 [J]). */
mg_status mgh_level_info(const mgh_ctx* ctx, int64_t* n);

/* Release the context.  Waits for its work.  NULL is ignored. */
void mgh_destroy(mgh_ctx* ctx);

/* Message describing the last failure on this thread ("" if none). */
const char* mgh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGH_H */
