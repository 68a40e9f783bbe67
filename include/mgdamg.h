/*
 * mgdamg — AMG block-preconditioned GMRES for the multi-group radiation
 * diffusion block system, on AMD Instinct MI355X (gfx950).
 *
 * Method: Yue, Zhang, Xu, Shu, Shi, "Algebraic multigrid block
 * preconditioning for multi-group radiation diffusion equations"
 * (arXiv 2002.04958).  Every numerical step runs in the library's own HIP
 * kernels; this header is the only boundary.
 *
 * Conventions
 *   - Pointers documented as [dev] are HIP device pointers on the context's
 *     device; [host] pointers are ordinary host memory.
 *   - Input arrays are borrowed for the duration of a call; everything a
 *     handle keeps is copied into memory the handle owns.  Output buffers
 *     are owned by the caller.
 *   - All device work is enqueued on the context's stream.  Calls whose
 *     result needs a host decision (setup, GMRES convergence) synchronise
 *     that stream before returning.
 *   - Every call returns MGD_OK (0) or a negative status; no exception or
 *     C++ type crosses this boundary.  mgd_last_error() gives a message for
 *     the last non-OK status of the calling thread.
 *   - Index arrays are int32 (sizes up to 2^31 - 1 entries); counts that can
 *     exceed that are int64.
 */
#ifndef MGDAMG_H
#define MGDAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mgd_status;
enum {
  MGD_OK = 0,
  MGD_EINVAL = -1,      /* invalid argument or structure; nothing was launched */
  MGD_ENOMEM = -2,      /* device allocation failed */
  MGD_EHIP = -3,        /* a HIP runtime call failed */
  MGD_ENOTCONV = -4,    /* iteration limit reached; outputs hold the last iterate */
  MGD_EBREAKDOWN = -5,  /* Krylov breakdown with a singular Hessenberg matrix */
  MGD_ESINGULAR = -6,   /* zero pivot in a coarsest-level factorisation */
  MGD_ESTATE = -7       /* handle used with the wrong context or after destroy */
};

/* Message for the last non-OK status returned on this thread. */
const char* mgd_last_error(void);
const char* mgd_version(void);

/* ---------------------------------------------------------------------------
 * Context: device, stream and allocator.
 *   device     HIP device ordinal; made current for every call on the context.
 *   hip_stream hipStream_t to enqueue on (NULL: the default stream).
 *   allocator  optional callbacks for all device memory the library owns
 *              (NULL: hipMalloc/hipFree).  alloc returns NULL on failure.
 * ------------------------------------------------------------------------- */
typedef struct mgd_ctx mgd_ctx;
typedef struct mgd_allocator {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} mgd_allocator;

mgd_status mgd_ctx_create(int device, void* hip_stream, const mgd_allocator* allocator,
                          mgd_ctx** out);
mgd_status mgd_ctx_destroy(mgd_ctx* ctx);
mgd_status mgd_ctx_synchronize(mgd_ctx* ctx);

/* Per-kernel-class timing.  When enabled, every launch of the library's
 * solve-phase kernels is bracketed by HIP events on the context stream and
 * its algorithmic HBM bytes (each matrix entry, index and vector element
 * counted once per launch) are accumulated per class.  Classes are named by
 * mgd_kernel_class_name(i), i = 0 .. mgd_kernel_class_count()-1.
 * mgd_ctx_kernel_stats synchronises the stream. */
mgd_status mgd_ctx_set_profiling(mgd_ctx* ctx, int enable);
mgd_status mgd_ctx_reset_kernel_stats(mgd_ctx* ctx);
int mgd_kernel_class_count(void);
const char* mgd_kernel_class_name(int cls);
mgd_status mgd_ctx_kernel_stats(mgd_ctx* ctx, int cls, int64_t* launches, double* total_ms,
                                double* total_bytes);
/* The same statistics per kernel symbol, for the launches that a profiling
 * scope times alone (the V-cycle kernels, SpMV and the block matvec).  Names
 * are the kernel's name with its template arguments as a demangler prints
 * them, e.g. "k_half<float, 1>", followed for V-cycle kernels by
 * "@L<level>/<hierarchies in the union>".  total_bytes counts the matrix in
 * its stored layout (e.g. 16-bit column offsets); total_bytes_csr prices the
 * same launches as plain CSR (value and 4-byte column per entry, 4-byte row
 * pointer per row swept; block matvec: the pattern once per block), vectors
 * alike.  mgd_ctx_kernel_symbol_count synchronises; name receives at most
 * name_cap-1 characters and a terminating zero; any output may be NULL. */
mgd_status mgd_ctx_kernel_symbol_count(mgd_ctx* ctx, int* count);
mgd_status mgd_ctx_kernel_symbol_stats(mgd_ctx* ctx, int index, char* name, int name_cap,
                                       int64_t* launches, double* total_ms, double* total_bytes,
                                       double* total_bytes_csr);

/* ---------------------------------------------------------------------------
 * Sparse matrices (CSR).  Columns sorted ascending within each row; every
 * square matrix handed to AMG stores its diagonal entry.  All arrays [dev].
 * ------------------------------------------------------------------------- */
typedef struct mgd_csr {
  int32_t n_rows, n_cols;
  int64_t nnz;
  const int32_t* row_ptr; /* [dev] n_rows + 1 */
  const int32_t* col_idx; /* [dev] nnz */
  const double* val;      /* [dev] nnz */
} mgd_csr;

/* y = A x.  x [dev] n_cols, y [dev] n_rows (must not alias x). */
mgd_status mgd_csr_spmv(mgd_ctx* ctx, const mgd_csr* A, const double* x, double* y);

/* ---------------------------------------------------------------------------
 * Classical AMG (Section 3.1 of the paper: strength threshold 0.25, V(1,1)
 * with C-then-F relaxation going down and F-then-C going up, classical
 * modified interpolation, Galerkin coarse operators with R = P^T, at most
 * 100 unknowns on the coarsest level solved by Gaussian elimination).
 * Coarsening is seeded PMIS (the paper's Falgout coarsening is sequential);
 * the smoother is CF-ordered l1-Jacobi.  Setup runs on the device.
 * ------------------------------------------------------------------------- */
typedef struct amg_params {
  double strength_theta;  /* 0.25 */
  double dominance_theta; /* 0.9: rows with row sum >= theta * a_ii have no strong
                             dependencies (Definition 2 threshold); <= 0 disables */
  uint64_t seed;          /* PMIS hash seed */
  int32_t max_levels;     /* 25 */
  int32_t coarse_max;     /* 100 */
  int32_t dense_max;      /* 2000: larger stalled coarsest levels are relaxed instead */
  int32_t n_pre, n_post;  /* 1, 1 */
  int32_t precision;      /* 0: FP64 solve phase; 1: FP32 matrices and vectors
                             (coarsest solve stays FP64) */
  int32_t autotune;       /* 1: time the residual kernel of every level matrix, and the
                             restriction kernel of every restriction, of at least 131072
                             rows in each candidate layout (sliced ELL; CSR with 1-32
                             lanes per row; 64, 128 or 256 threads per workgroup), keep
                             the fastest unless the default layout is within 3% of it,
                             and cache the choice per (role, rows, nnz, longest row) in
                             the process and, when the environment names one, in the
                             file MGD_AUTOTUNE_CACHE; smaller matrices keep the default
                             layouts.  The layout changes which lanes add a row's
                             entries, so results may differ from the default layouts'
                             in rounding. */
  int32_t coarsening;     /* 0: PMIS; 1: HMIS (Ruge-Stueben first pass inside tiles of
                             hmis_tile consecutive rows, then PMIS for the rest) */
  int32_t hmis_tile;      /* 1024, in [1, 1024] */
  int32_t smoother;       /* 0: CF-ordered l1-Jacobi; 1: multicolour Gauss-Seidel (Jones-
                             Plassmann colours, ascending going down, descending going up;
                             a stalled coarsest level is relaxed the same way) */
  int32_t aggressive_levels; /* 0: the number of finest levels coarsened aggressively
                                (Section 3.1 uses 1): a second pass of the same coarsening
                                over the C points on their strength graph of distance two,
                                with multipass interpolation; in [0, MGD_MAX_LEVELS] */
} amg_params;
void amg_params_default(amg_params* p);

typedef struct amg_hierarchy amg_hierarchy;

/* Build a hierarchy for the square matrix A.  The matrix is copied. */
mgd_status amg_setup(mgd_ctx* ctx, const mgd_csr* A, const amg_params* p, amg_hierarchy** out);

/* z = k V-cycles applied to r from a zero initial guess
 * (z <- z + V(r - A z)).  r, z [dev] length n; must not alias. */
mgd_status amg_apply(mgd_ctx* ctx, amg_hierarchy* h, const double* r, double* z, int n_cycles);

#define MGD_MAX_LEVELS 32
typedef struct amg_info {
  int32_t levels;
  int32_t coarse_kind;          /* 0: dense LU, 1: l1-Jacobi sweeps (stalled) */
  int64_t n[MGD_MAX_LEVELS];
  int64_t nnz[MGD_MAX_LEVELS];
  int64_t nnz_P[MGD_MAX_LEVELS]; /* P_l: n[l] x n[l+1]; 0 on the coarsest level */
  int32_t pmis_rounds[MGD_MAX_LEVELS];
  double grid_complexity;
  double operator_complexity;
} amg_info;
mgd_status amg_get_info(const amg_hierarchy* h, amg_info* out);

/* Copy level data to host buffers sized from amg_info (any may be NULL):
 * cf (n[l]: 1 = C, -1 = F; all -1... undefined on the coarsest level),
 * the level matrix A_l (n[l]+1, nnz[l], nnz[l]) and P_l (n[l]+1, nnz_P[l]).
 * Level matrices are reported in their natural (setup) ordering. */
mgd_status amg_export_level(mgd_ctx* ctx, const amg_hierarchy* h, int level, int8_t* cf,
                            int32_t* a_row_ptr, int32_t* a_col, double* a_val,
                            int32_t* p_row_ptr, int32_t* p_col, double* p_val);
mgd_status amg_destroy(amg_hierarchy* h);

/* ---------------------------------------------------------------------------
 * The block system of eq. 2.2: G+2 diagonal blocks ordered [1..G, E, I] on a
 * common cell numbering of size N, and diagonal couplings.  Unknowns of the
 * monolithic vector are ordered [T_1 .. T_G, T_E, T_I], each a segment of N.
 * ------------------------------------------------------------------------- */
typedef struct mgd_block_system {
  int32_t G;
  int32_t N;
  const mgd_csr* blocks; /* [host] array of G+2 matrices (their arrays [dev]) */
  const double* d_gE;    /* [dev] G*N: diagonal of D_gE, row g, column E */
  const double* d_Eg;    /* [dev] G*N: diagonal of D_Eg, row E, column g */
  const double* d_EI;    /* [dev] N */
  const double* d_IE;    /* [dev] N */
} mgd_block_system;

/* y = A x with the block form of eq. 2.2.  x, y [dev] (G+2)*N, no aliasing. */
mgd_status mgd_block_matvec(mgd_ctx* ctx, const mgd_block_system* A, const double* x, double* y);

/* Per-cell coefficients of the cell-centred discretisation: n^dim unit
 * cells (x-fastest), harmonic face means 2 k_a k_b / (k_a + k_b) on interior
 * faces, zero-flux boundary, mass term on every diagonal, couplings
 * D_gE = -c_gE, D_Eg = -c_Eg, D_EI = D_IE = -c_EI each also added to the
 * diagonal of its row.  xi (optional) scales the off-diagonal of row i in
 * face direction d (-x,+x,-y,+y,-z,+z) by (1 + 0.5 xi) for a nonsymmetric
 * variant. */
typedef struct mgd_coeffs {
  int32_t dim, n, G;
  const double* kappa; /* [dev] (G+2)*N */
  const double* c_gE;  /* [dev] G*N */
  const double* c_Eg;  /* [dev] G*N */
  const double* c_EI;  /* [dev] N */
  double mass;
  const double* xi;    /* [dev] (G+2)*N*2*dim or NULL */
} mgd_coeffs;

/* Assemble eq. 2.2 on the device into library-owned arrays; release with
 * mgd_block_system_free.  The arrays are read-only for the caller: when every
 * block equals its transpose bit for bit (xi == NULL), the library also keeps
 * each block's values on and above the diagonal for the block matvec (the
 * entries below read their mirrors'; same results bit for bit), freed with the
 * system. */
mgd_status mgd_assemble(mgd_ctx* ctx, const mgd_coeffs* c, mgd_block_system* out);
/* A^T as a block system (blocks transposed, D_gE and D_Eg swapped, D_EI and
 * D_IE swapped), library-owned and read-only like an assembled one (with the
 * same half storage when its blocks share one pattern and are symmetric). */
mgd_status mgd_block_system_transpose(mgd_ctx* ctx, const mgd_block_system* A,
                                      mgd_block_system* out);
mgd_status mgd_block_system_free(mgd_ctx* ctx, mgd_block_system* s);

/* ---------------------------------------------------------------------------
 * Block preconditioners (Section 3).  apply computes z = M^{-1} r.
 *   AMG_MONO     one hierarchy on the monolithic matrix (Section 3.1)
 *   BLOCK_DIAG   A_1..A_G, A_E, A_I inverted independently (Section 3.5 remark)
 *   PCTL         block relaxation E, then groups and I, then the coarse
 *                correction with A_c of eq. 3.1 (Section 3.2); the diagonal
 *                interpolation weights come from V-cycles run to pctl_p_tol
 *   SCHUR1       five steps with C^_E, C^_g and A_I (Sections 3.3, 3.4)
 *   SCHUR2       three steps with A_E, S^_g and S^_I (Sections 3.3, 3.4)
 *   SCHUR2_LOWER Schur2 steps 1-2: the elimination factor of eq. 3.3
 *   IDENTITY     z = r
 * Each scalar inverse is a fixed number of V-cycles (option #2 of Section
 * 3.4): cycles_rad for group blocks, cycles_E for E blocks (and A_c),
 * cycles_I for I blocks.  batched = 1 applies the independent V-cycles of a
 * step (the group blocks, plus I where the step has it) as one set of
 * launches over all hierarchies; use_graph = 1 replays the whole apply from
 * a captured HIP graph.  transpose = 1 builds the preconditioner on A^T.
 *
 * adaptive = 1 (PCTL, SCHUR1, SCHUR2: the alpha-variants of Section 3.5)
 * forms the preconditioner from the system with its weak couplings
 * neglected: a coupling block D_ab is weak when more than sigma_wc N of its
 * rows have -d_kk <= theta_wc a_kk, a_kk the diagonal of the row block A_a
 * (Definition 1).  A row block whose coupling to E is neglected is solved
 * independently of E; when every row block's coupling to E is neglected the
 * two E inverses of Schur1/Schur2 become one after the independent solves,
 * and when every coupling in E's row is neglected the E correction step (and
 * PCTL's coarse-grid correction) is skipped.  Each scalar inverse whose
 * matrix has no row with sum_j a_kj < theta_wd a_kk (Definition 2) uses
 * jacobi_sweeps Jacobi iterations from zero (option #1 of Section 3.4)
 * instead of V-cycles; PCTL's interpolation weights keep option #3.
 *
 * inner_tol > 0 approximates the inverses that the paper's experiments solve
 * to a relative tolerance (Section 4; option #3 of Section 3.4) by V-cycles
 * z <- z + V(r), r = b - A z, until ||r|| < inner_tol ||b|| or
 * inner_maxcycles cycles: the hatted matrices of SCHUR1 (C^_E, C^_g) and
 * SCHUR2/SCHUR2_LOWER (S^_g, S^_I) and PCTL's block relaxations (A_E, A_g,
 * A_I); the other inverses keep their fixed cycle counts.  In a batched step
 * each member stops on its own criterion.  The preconditioner is then
 * nonlinear (use flexible GMRES) and every apply synchronises once per inner
 * cycle, so use_graph is ignored.
 *
 * option4_steps > 0 (SCHUR2, SCHUR1; option #4 of Section 3.4) replaces the
 * hatted S^_I^{-1} of Schur2 (C^_E^{-1} of Schur1) by that many steps from
 * zero of w <- A_I^{-1}(q + D_IE A_E^{-1}(D_EI w))  (Schur1: E and I
 * exchanged), with the original blocks' inverses inside; the I hierarchy of
 * Schur2 (E hierarchy of Schur1) is then built on the original block.
 * ------------------------------------------------------------------------- */
enum {
  MGD_PC_AMG_MONO = 0,
  MGD_PC_BLOCK_DIAG = 1,
  MGD_PC_PCTL = 2,
  MGD_PC_SCHUR1 = 3,
  MGD_PC_SCHUR2 = 4,
  MGD_PC_SCHUR2_LOWER = 5,
  MGD_PC_IDENTITY = 6
};

typedef struct block_params {
  int32_t kind;
  amg_params amg;
  int32_t cycles_rad, cycles_E, cycles_I; /* 1, 1, 1 */
  double pctl_p_tol;                      /* 1e-2 */
  int32_t pctl_p_maxcycles;               /* 100 */
  int32_t batched;                        /* 0 sequential launches, 1 batched */
  int32_t use_graph;                      /* 0 / 1 */
  int32_t transpose;                      /* 0 / 1 */
  int32_t adaptive;                       /* 0 / 1 (PCTL, SCHUR1, SCHUR2) */
  double theta_wc;                        /* 1e-2, Definition 1 */
  double sigma_wc;                        /* 0.5 */
  double theta_wd;                        /* 0.9, Definition 2 */
  int32_t jacobi_sweeps;                  /* 2, option #1 */
  double inner_tol;                       /* 0 = fixed cycles (option #2); 1e-2 in Section 4 */
  int32_t inner_maxcycles;                /* 100 */
  int32_t option4_steps;                  /* 0 = hatted inverse; > 0 option #4 */
} block_params;
void block_params_default(block_params* p);

typedef struct block_precond block_precond;
mgd_status block_precond_create(mgd_ctx* ctx, const mgd_block_system* A, const block_params* p,
                                block_precond** out);
/* r, z [dev] (G+2)*N, no aliasing. */
mgd_status block_precond_apply(mgd_ctx* ctx, block_precond* M, const double* r, double* z);

typedef struct block_precond_info {
  int32_t kind;
  int32_t n_hierarchies;
  int32_t inverses_per_apply;   /* scalar inverses (V-cycle sets) per apply */
  int32_t matvecs_per_apply;    /* block SpMVs per apply (PCTL step 2) */
  int32_t pctl_p_cycles[66];    /* V-cycles used for p_1..p_G, p_I */
  double setup_ms;
  /* adaptive = 1 only (zero otherwise): Definition 1 counts and the
   * neglected couplings, Definition 2 counts per inverse role (g < G, G: E,
   * G+1: I; -1 where not evaluated) and the roles that use Jacobi */
  int32_t wc_count_gE[64], wc_count_Eg[64], wc_count_EI, wc_count_IE;
  uint8_t weak_gE[64], weak_Eg[64];
  int32_t weak_EI, weak_IE;
  int32_t wd_count[66];
  uint8_t jacobi[66];
  /* inner_tol > 0: V-cycles each inverse role used in the last apply (-1 for
   * roles with a fixed cycle count) */
  int32_t inner_cycles[66];
} block_precond_info;
mgd_status block_precond_get_info(const block_precond* M, block_precond_info* out);
/* Hierarchy of one scalar inverse: index g < G for group g, G for the E
 * block (A_E, C^_E), G+1 for the I block, G+2 for the PCTL coarse matrix;
 * 0 for AMG_MONO.  The handle stays owned by M. */
mgd_status block_precond_get_hierarchy(const block_precond* M, int index,
                                       const amg_hierarchy** out);
mgd_status block_precond_destroy(block_precond* M);

/* ---------------------------------------------------------------------------
 * Restarted GMRES(m) with right preconditioning (the paper's outer solver,
 * Section 2 and Section 4): Arnoldi with classical Gram-Schmidt applied
 * twice, Givens rotations, stop when the residual estimate is <= rtol ||b||
 * and the true residual confirms it.  flexible = 1 stores M^{-1} v_j (FGMRES);
 * flexible = 0 forms x += M^{-1}(V y) once per cycle.
 * ------------------------------------------------------------------------- */
typedef struct gmres_params {
  int32_t restart;   /* 30 */
  int32_t max_iters; /* 1000 */
  double rtol;       /* 1e-8 */
  int32_t flexible;  /* 1 */
  int32_t profile;   /* 1: fill the per-phase times of gmres_result */
} gmres_params;
void gmres_params_default(gmres_params* p);

typedef struct gmres_result {
  int32_t iters;      /* Arnoldi steps over all cycles */
  int32_t restarts;   /* completed cycles */
  int32_t converged;
  int32_t precond_applies;
  double relres_est;  /* |g_{j+1}| / ||b|| at exit */
  double relres_true; /* ||b - A x|| / ||b|| at exit */
  double t_total_ms;
  double t_precond_ms, t_matvec_ms, t_orth_ms; /* when profile = 1 */
  int32_t reorths;    /* Arnoldi steps that needed the second Gram-Schmidt pass */
} gmres_result;

/* Solve A x = b.  x [dev] holds the initial guess on entry.  M may be NULL
 * (no preconditioning).  Returns MGD_ENOTCONV when max_iters is reached. */
mgd_status gmres_solve(mgd_ctx* ctx, const mgd_block_system* A, block_precond* M,
                       const double* b, double* x, const gmres_params* p, gmres_result* out);

/* gmres_solve for callers that cannot allocate device memory (work under
 * HIP graph capture around the call, serving loops, harnesses that forbid
 * hipMalloc): the same arguments, iteration and result as gmres_solve, with
 * no device allocation, no pinned host allocation and no graph instantiation.
 * The Krylov basis V ((m+1) n doubles), the preconditioned vectors Z (m n,
 * flexible with a preconditioner) or two n-vectors (non-flexible), the
 * Hessenberg scratch and the reduction partials (about 0.5 MiB) live in a
 * static device array of 64 MiB per device, held until the process ends;
 * n = (G+2) N, m = restart.  Sizes that do not fit return MGD_EINVAL before
 * any launch (with m = 30 and a flexible preconditioned solve, up to about
 * 137,000 unknowns); profile = 1 returns MGD_EINVAL.  Preconditioner applies
 * run as direct launches (a use_graph preconditioner is not replayed here)
 * and the whole solve stays on the context stream.  Every call on one device
 * shares that device's array and leaves its contents behind: calls that
 * overlap on one device race, so run them on one stream or one at a time.
 * M must have been created (its own memory allocated) beforehand. */
mgd_status gmres_solve_noalloc(mgd_ctx* ctx, const mgd_block_system* A, block_precond* M,
                               const double* b, double* x, const gmres_params* p,
                               gmres_result* out);

/* ---------------------------------------------------------------------------
 * Adjoint.  With A x = b and g = dL/dx: solve A^T lambda = g by GMRES with
 * M_T (a preconditioner created with transpose = 1 on A), then
 *   dL/db = lambda
 *   dL/dkappa[a][c] = sum over faces f of c: -(lam_c - lam_nb)(x_c - x_nb)
 *                      * 2 kappa_nb^2 / (kappa_c + kappa_nb)^2
 *   dL/dc_gE = -lam_g (x_g - x_E), dL/dc_Eg = -lam_E (x_E - x_g),
 *   dL/dc_EI = -lam_E (x_E - x_I) - lam_I (x_I - x_E)
 * dL_dkappa [dev] (G+2)*N or NULL; dL_dc [dev] (2G+1)*N ordered
 * [c_gE (G*N), c_Eg (G*N), c_EI (N)] or NULL.  Defined for xi == NULL.
 * ------------------------------------------------------------------------- */
mgd_status adjoint_solve(mgd_ctx* ctx, const mgd_coeffs* c, const mgd_block_system* A,
                         block_precond* M_T, const double* x, const double* g, double* lambda,
                         double* dL_dkappa, double* dL_dc, const gmres_params* p,
                         gmres_result* out);
/* The gradient step alone, for given x and lambda. */
mgd_status mgd_adjoint_gradients(mgd_ctx* ctx, const mgd_coeffs* c, const double* x,
                                 const double* lambda, double* dL_dkappa, double* dL_dc);

#ifdef __cplusplus
}
#endif
#endif /* MGDAMG_H */
