/*
 * nnmg.h -- C ABI of the matrix-free non-nested multigrid library for gfx950.
 *
 * The library solves continuous Lagrange Q_k (k = 1..4) finite-element Poisson
 * problems -Laplace(u) = f with homogeneous Dirichlet conditions on
 * quadrilateral (d = 2) and hexahedral (d = 3) meshes, using a multigrid
 * preconditioner whose levels are independent, non-nested meshes of the same
 * domain (paper §2, "Non-nested multigrid method").
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every int-returning call returns NNMG_OK (0) or a negative
 *   NNMG_ERR_* code; nnmg_last_error() returns a thread-local message for the
 *   last failure.  No C++ exception crosses this boundary.  Output handles are
 *   written only on success; destroy(NULL) is a no-op.
 * - Meshes are host arrays, copied during *_create.  Vertices: float64
 *   [n_vertices][dim].  Cells: int32 [n_cells][2^dim]; local vertex b of a cell
 *   sits at the reference corner whose coordinate along axis a is bit a of b
 *   (x fastest).  Cells must be positively oriented.  dirichlet_vertex: uint8
 *   [n_vertices] or NULL (no Dirichlet boundary).
 * - A DoF is constrained (fixed to zero) iff it lies on the closure of a
 *   boundary face whose vertices are all flagged Dirichlet.
 * - Vectors are device pointers of length n_dofs (all DoFs, constrained
 *   included) in the library's DoF numbering, contiguous, on the context's
 *   device, float64 for NNMG_FP64 and float32 for NNMG_FP32.  Constrained
 *   entries of right-hand sides and residuals must be zero.  Input and output
 *   vectors of one call must not alias.
 * - Streams are hipStream_t values passed as void* (NULL = default stream).
 *   vmult, prolongate, restrict and vcycle are asynchronous on that stream;
 *   *_create, pcg_solve and the query calls are synchronous.
 * - A hierarchy is not re-entrant: calls on one hierarchy must not overlap.
 *   Different hierarchies may run concurrently on different streams.
 * - Transfers and hierarchies keep references to their levels, so handles may
 *   be destroyed in any order.
 */
#ifndef NNMG_H
#define NNMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NNMG_OK = 0,
    NNMG_ERR_INVALID_ARG = -1,     /* bad pointer, size, dimension or option */
    NNMG_ERR_UNSUPPORTED = -2,     /* degree outside 1..4, dim outside 2..3 */
    NNMG_ERR_OOM = -3,             /* a device allocation failed */
    NNMG_ERR_MESH = -4,            /* invalid mesh (index range, inverted cell) */
    NNMG_ERR_POINT_NOT_FOUND = -5, /* a fine point has no coarse owner cell */
    NNMG_ERR_NOT_CONVERGED = -6,   /* CG hit max_it before the tolerance */
    NNMG_ERR_BREAKDOWN = -7,       /* NaN or non-positive curvature in CG */
    NNMG_ERR_HIP = -8              /* a HIP runtime call failed */
};

typedef enum { NNMG_FP64 = 0, NNMG_FP32 = 1 } nnmg_prec;

typedef struct nnmg_ctx nnmg_ctx;
typedef struct nnmg_level nnmg_level;
typedef struct nnmg_transfer nnmg_transfer;
typedef struct nnmg_hierarchy nnmg_hierarchy;

/* Device memory provider.  alloc returns a device pointer of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  A NULL allocator in
 * nnmg_ctx_create means hipMalloc / hipFree. */
typedef struct {
    void* user;
    void* (*alloc)(void* user, size_t bytes, void* stream);
    void (*free)(void* user, void* ptr, void* stream);
} nnmg_allocator;

typedef struct {
    int dim;                         /* 2 or 3 */
    int64_t n_vertices;
    const double* vertices;          /* host [n_vertices][dim] */
    int64_t n_cells;
    const int32_t* cells;            /* host [n_cells][2^dim] */
    const uint8_t* dirichlet_vertex; /* host [n_vertices] or NULL */
} nnmg_mesh;

/* Point location settings of nnmg_transfer_create (paper §3.1 and §3.3). */
typedef struct {
    double bbox_expand;   /* candidate cells: vertex bounding box grown on every side by
                             bbox_expand times its diagonal (default 0.25) */
    double inside_tol;    /* a pre-image within this max-norm distance of [0,1]^d is
                             inside the cell (default 1e-10) */
    double newton_tol;    /* Newton stops when the update's max-norm is <= this (1e-12) */
    int newton_max_it;    /* Newton gives up after this many steps (default 50) */
    int allow_projection; /* 1: points outside every candidate are projected onto the
                             nearest candidate's reference cell (eq. closest_point);
                             0: such points are an error (default 1) */
    int nested_p;         /* 1 (default): when both levels have the same mesh (vertices and
                             cells) and the coarse degree is lower, the transfer is the nested
                             polynomial one (paper §2, Coarse grid solvers): no point location,
                             sum-factorized interpolation per cell; 0: always locate points */
} nnmg_transfer_opts;

/* Multigrid settings of nnmg_hierarchy_create (paper §4 solver recipe). */
typedef struct {
    int cheb_degree;          /* Chebyshev degree per smoothing sweep (default 3) */
    double smoothing_range;   /* interval [lambda_max / range, lambda_max] (default 20) */
    double eig_safety;        /* lambda_max = safety * Lanczos estimate (default 1.2) */
    int eig_iters;            /* Lanczos (Jacobi-CG) steps (default 12) */
    const void* const* eig_start; /* NULL, or one entry per level (coarse -> fine): a float64
                                     device vector [n_dofs] used as the Lanczos start vector,
                                     or NULL for the library's seeded SplitMix64 vector */
} nnmg_mg_opts;

/* Settings of nnmg_pcg_solve. */
typedef struct {
    double rtol;            /* stop when ||r_k||_2 <= rtol ||b||_2 (default 1e-8) */
    int max_it;             /* iteration limit (default 200) */
    nnmg_prec vcycle_prec;  /* precision of the V-cycle preconditioner (default FP32) */
    double* history;        /* host [max_it + 1] or NULL: ||r_k||_2 / ||b||_2, k = 0.. */
    int use_graph;          /* 1 (default): the preconditioner V-cycle is captured once per
                               precision as a HIP graph and replayed every iteration (bitwise
                               the same arithmetic as launching it kernel by kernel, 0);
                               the graph is rebuilt after nnmg_set_cheb_bounds, and not used
                               while profiling is on */
} nnmg_cg_opts;

/* The operator of a level. */
typedef enum {
    NNMG_OP_LAPLACE = 0,    /* -div grad u (paper §2, eq. problem) */
    NNMG_OP_ELASTICITY = 1  /* linear elasticity, -div sigma(u) (paper §4, Applications to FEA,
                               eq. linear_elasticity): vector Q_k with dim components, 3D only */
} nnmg_operator;

/* Settings of nnmg_level_create_ex. */
typedef struct {
    nnmg_operator op;  /* default NNMG_OP_LAPLACE */
    double lambda;     /* Lame coefficients of NNMG_OP_ELASTICITY (default 1, 1); */
    double mu;         /* sigma = lambda tr(eps) I + 2 mu eps, mu > 0, lambda >= 0 */
} nnmg_level_opts;

typedef struct {
    int iterations;  /* CG iterations performed */
    double relres;   /* final ||r||_2 / ||b||_2 */
    int status;      /* NNMG_OK, NNMG_ERR_NOT_CONVERGED or NNMG_ERR_BREAKDOWN */
} nnmg_cg_result;

/* ------------------------------------------------------------------------ */
/* Context and error reporting                                               */
/* ------------------------------------------------------------------------ */

/* Binds the library to HIP device `device`.  allocator may be NULL. */
int nnmg_ctx_create(int device, const nnmg_allocator* allocator, nnmg_ctx** out);
void nnmg_ctx_destroy(nnmg_ctx* ctx);
/* Message of the last failing call on this thread ("" if none). */
const char* nnmg_last_error(void);

void nnmg_default_level_opts(nnmg_level_opts* opts);
void nnmg_default_transfer_opts(nnmg_transfer_opts* opts);
void nnmg_default_mg_opts(nnmg_mg_opts* opts);
void nnmg_default_cg_opts(nnmg_cg_opts* opts);

/* ------------------------------------------------------------------------ */
/* Levels (paper §2: one mesh T_l and its space V_l with Q^p elements)       */
/* ------------------------------------------------------------------------ */

/* Sets up one level: DoF numbering (Gauss-Lobatto support points), the
 * cell-to-DoF map, the constrained set, the geometry at the (k+1)^d Gauss
 * points (paper §4) and the inverse Jacobi diagonal.  Synchronous.
 * The operator starts in variant 0 (nnmg_level_tune) with one layout block
 * per workgroup in both precisions, unless the environment at creation asks
 * otherwise: NNMG_GEOMETRY=metric (stored metric), NNMG_SCATTER=atomic (float
 * atomics), NNMG_SWEEP=transposed (transposed sweeps), NNMG_INDEX=entity
 * (entity-compressed indices, 3D Laplace, degree >= 3); NNMG_CELL_ORDER=input
 * keeps the cell blocks in input order instead of the Morton order of their
 * centroids.  All of them give the same operator up to the order of
 * floating-point sums.
 * Errors: UNSUPPORTED (degree or dim), INVALID_ARG, MESH (vertex index out
 * of range, repeated vertex in a cell, non-positive Jacobian at a Gauss
 * point), OOM, HIP. */
int nnmg_level_create(nnmg_ctx* ctx, const nnmg_mesh* mesh, int degree, nnmg_level** out);

/* As nnmg_level_create, with the operator chosen by opts (NULL: defaults).
 * For NNMG_OP_ELASTICITY (paper §4, Applications to FEA) a level carries
 * dim displacement components per Q_k node; every vector of the level has
 * n_dofs = dim * n_nodes entries interleaved by node (component c of node i
 * at dim * i + c).  The clamped boundary is the union of the faces whose
 * vertices all carry the Dirichlet flag (all components fixed at zero there);
 * every other boundary face is traction free.  Transfers and hierarchies
 * accept elasticity levels like Laplace levels (P acts on each component).
 * Errors as nnmg_level_create; UNSUPPORTED for elasticity in 2D; INVALID_ARG
 * for mu <= 0 or lambda < 0. */
int nnmg_level_create_ex(nnmg_ctx* ctx, const nnmg_mesh* mesh, int degree, const nnmg_level_opts* opts,
                         nnmg_level** out);
void nnmg_level_destroy(nnmg_level* level);

/* n_dofs: entries of the level's vectors (ncomp * nodes); n_free: those not
 * constrained. */
int nnmg_level_info(const nnmg_level* level, int64_t* n_dofs, int64_t* n_free, int64_t* n_cells);

/* Components per node: 1 (Laplace) or dim (elasticity). */
int nnmg_level_components(const nnmg_level* level, int* ncomp);

/* Support point of every DoF: host [n_dofs][dim] (paper §2, eq. pointwise);
 * the components of one node share its point. */
int nnmg_level_support_points(const nnmg_level* level, double* host_xyz);

/* Constrained flag of every DoF: host uint8 [n_dofs]. */
int nnmg_level_constrained(const nnmg_level* level, uint8_t* host_mask);

/* Physical Gauss points: host [n_cells][(k+1)^dim][dim], cells in input order,
 * points lexicographic (x fastest). */
int nnmg_level_quadrature_points(const nnmg_level* level, double* host_xyz);

/* b_i = sum over cells and Gauss points of f_q phi_i(x_q) |det J_q| w_q
 * (paper §2: the load functional b(v) of eq. problem, with the Gauss rule of
 * §4).  f_qp_dev: float64 device [n_cells][(k+1)^dim][ncomp] values of f at
 * the points of nnmg_level_quadrature_points (for elasticity the body force,
 * b_(i,c) = sum f_c phi_i |det J| w).  b_dev is overwritten; its constrained
 * entries are zero.  Asynchronous on `stream`. */
int nnmg_level_assemble_rhs(nnmg_level* level, const double* f_qp_dev, double* b_dev, void* stream);

/* dst = A_l src by sum factorisation (paper §3.2: tensor-product evaluation at
 * Gauss points; the operator of eq. linear_system).  Constrained rows are the
 * identity (dst_c = src_c); constrained entries of src do not enter the
 * unconstrained rows.  src and dst must not alias.  Asynchronous. */
int nnmg_vmult(const nnmg_level* level, nnmg_prec prec, const void* src_dev, void* dst_dev, void* stream);

/* nnmg_vmult for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result, computed by the same kernels in the same order (the
 * deterministic contribution-slot path, whatever variant the level is tuned
 * to, where nnmg_vmult takes the slot path), with the per-(cell, node)
 * contribution slots kept in one static device
 * array of 64 MiB per GPU (held from the library's loading until the process
 * ends) instead of the level's own buffer.  The call allocates nothing and
 * calls no allocating routine.  Arguments as for nnmg_vmult (one right-hand
 * side).  Errors: NNMG_ERR_UNSUPPORTED when the level's slots need more than
 * 64 MiB in this precision (slots x components x 8 or 4 bytes; use
 * nnmg_vmult), NNMG_ERR_INVALID_ARG as for nnmg_vmult.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (unordered streams
 * or threads) race and must be serialised by the caller.  Asynchronous. */
int nnmg_vmult_noalloc(const nnmg_level* level, nnmg_prec prec, const void* src_dev, void* dst_dev, void* stream);

/* dst += A_l src restricted to the unconstrained rows and columns: the cell
 * loop of nnmg_vmult alone (constrained entries of src are read as zero and
 * constrained entries of dst are left unchanged).  One kernel launch; used to
 * accumulate several operator applications into one vector.  src and dst must
 * not alias.  Asynchronous. */
int nnmg_vmult_add(const nnmg_level* level, nnmg_prec prec, const void* src_dev, void* dst_dev, void* stream);

/* Several right-hand sides.  The _multi calls apply the operation of their
 * single-vector counterpart to nrhs vectors (1 <= nrhs <= 8) at once, in one
 * set of launches that reads the level's indices and geometry once for all of
 * them.  Vectors are interleaved: entry i of right-hand side r is element
 * i * nrhs + r of a [n_dofs][nrhs] array (n_dofs * nrhs entries).  Each
 * right-hand side gets exactly the arithmetic of a single-vector call.  The
 * first call with a larger nrhs than before grows the object's internal
 * buffers and synchronizes the device.  Errors: INVALID_ARG for nrhs out of
 * range, as the single-vector calls otherwise. */
int nnmg_vmult_multi(const nnmg_level* level, nnmg_prec prec, int nrhs, const void* src_dev, void* dst_dev,
                     void* stream);
int nnmg_vmult_add_multi(const nnmg_level* level, nnmg_prec prec, int nrhs, const void* src_dev, void* dst_dev,
                         void* stream);

/* Diagonal of A_l (1 on constrained rows) into diag_dev.  Asynchronous. */
int nnmg_level_diagonal(const nnmg_level* level, nnmg_prec prec, void* diag_dev, void* stream);

/* ------------------------------------------------------------------------ */
/* Non-nested transfer between two levels (paper §2 eq. residual2; §3)        */
/* ------------------------------------------------------------------------ */

/* Locates every unconstrained fine support point in the coarse mesh: bucket
 * grid over the grown coarse-cell boxes, Newton inversion of the trilinear
 * cell map, owner = lowest-numbered cell containing the point, otherwise
 * projection onto the nearest reference cell (eq. closest_point); stores the
 * points grouped by owner cell with their clamped reference coordinates
 * (the grouping runs on up to eight host threads for more than 2^20 points).
 * opts may be NULL (defaults).  Synchronous (timed setup).
 * Errors: INVALID_ARG (dim/device mismatch), POINT_NOT_FOUND, OOM, HIP. */
int nnmg_transfer_create(nnmg_ctx* ctx, const nnmg_level* fine, const nnmg_level* coarse,
                         const nnmg_transfer_opts* opts, nnmg_transfer** out);
void nnmg_transfer_destroy(nnmg_transfer* transfer);

/* Location results, in the order of the unconstrained fine DoFs:
 * fine_dof_host int32 [n_points] (may be NULL), owner_host int32 [n_points]
 * (may be NULL), xi_host float64 [n_points][dim] (may be NULL).  n_points and
 * n_projected may be NULL. */
int nnmg_transfer_points(const nnmg_transfer* transfer, int64_t* n_points, int32_t* fine_dof_host,
                         int32_t* owner_host, double* xi_host, int64_t* n_projected);

/* fine += P coarse, P_ij = phi_j^{coarse}(x_i) (paper §2 after eq. residual2;
 * §3.2 eqs. local_evaluation and tensor_product_evaluation).  Only
 * unconstrained fine entries change; constrained coarse entries are read as
 * zero.  Asynchronous. */
int nnmg_prolongate(const nnmg_transfer* transfer, nnmg_prec prec, const void* coarse_dev,
                    void* fine_dev_add, void* stream);

/* coarse += P^T fine (paper §2, eq. residual2): per coarse cell the sums over
 * its points go to slots sorted by coarse DoF, which are then added in a fixed
 * order (deterministic, no float atomics).  Only unconstrained coarse entries
 * change.  Uses the transfer's own slot buffer: calls on one transfer must not
 * overlap.  Asynchronous. */
int nnmg_restrict(const nnmg_transfer* transfer, nnmg_prec prec, const void* fine_dev,
                  void* coarse_dev_add, void* stream);

/* nnmg_prolongate / nnmg_restrict for nrhs interleaved right-hand sides (see
 * nnmg_vmult_multi for the layout and the limits). */
int nnmg_prolongate_multi(const nnmg_transfer* transfer, nnmg_prec prec, int nrhs, const void* coarse_dev,
                          void* fine_dev_add, void* stream);
int nnmg_restrict_multi(const nnmg_transfer* transfer, nnmg_prec prec, int nrhs, const void* fine_dev,
                        void* coarse_dev_add, void* stream);

/* ------------------------------------------------------------------------ */
/* Autotuner: kernel variants timed on the GPU at hand                          */
/* ------------------------------------------------------------------------ */

/* Timings of the variants of an operation and the one kept. */
typedef struct {
    int n_variants;  /* entries of ms that were timed */
    double ms[16];   /* average milliseconds per call of each variant, -1 where not timed */
    int chosen;      /* index of the variant now in use */
    int rhs_split;   /* nnmg_level_tune: several right-hand sides run one grid row each (1) or
                        every block loops over them (0) */
    double ms_rhs[2]; /* nnmg_level_tune: milliseconds of the 4-right-hand-side product looping (0) and
                         split (1), timed on small levels only (-1 otherwise) */
    int cells_per_block; /* nnmg_level_tune: cells per workgroup of the operator kept */
    double ms_cpb[2];    /* nnmg_level_tune: milliseconds of the variant kept with one (0) and two (1)
                            layout blocks per workgroup (-1 where not timed); ms[v] is the faster of
                            the two for each variant v */
} nnmg_tune_result;

/* Times the variants of the level's operator application in precision `prec`
 * as the V-cycle uses it (product and the residual that consumes it, reps
 * calls each after two warm-up calls, on a private stream) and keeps the
 * fastest for that precision; each precision has its own variant:
 *   0 geometry rebuilt from the trilinear map, contributions in slots
 *   1 geometry rebuilt from the trilinear map, float atomics
 *   2 stored merged metric per Gauss point,    contributions in slots
 *   3 stored merged metric per Gauss point,    float atomics
 *   4 as 0, with entity-compressed indices: per cell one record of the first
 *     DoF, first contribution slot, writer count and orientation of each of
 *     its 27 mesh entities instead of one DoF index and one slot per node
 *   5 as 2, with entity-compressed indices
 *   6..11 as 0..5 with transposed sweeps: between the contraction stages the
 *     lanes of a cell swap the line they own (x, y, z lines) through LDS, so
 *     every 1D contraction runs in registers (7 and 9 do not exist)
 * (variants 4, 5, 10 and 11 exist for 3D Laplace levels of degree >= 3,
 * otherwise NNMG_ERR_UNSUPPORTED; the elasticity operator has variant 0
 * only).  The variants differ only in the order of floating-point sums
 * (atomics: an order that varies between runs), the operator being the one of
 * paper §3.2 throughout.  Only the deterministic variants (0, 2, 4, 5, 6, 8,
 * 10, 11) are timed, so a
 * tuned level stays bitwise reproducible; the others keep ms = -1 and are
 * taken only when forced.  The stored metric is computed when a precision
 * needs it and freed when none does.  Each variant is timed with one and
 * with two layout blocks per workgroup (nnmg_level_set_cells_per_block), in
 * two passes over the candidates (the second in reverse order, the times
 * averaged, so that a drift of the clocks favours none), and the fastest pair
 * is kept (ms[v]: the faster of the two; ms_cpb: both, for
 * the variant kept); on small levels the two forms of several right-hand
 * sides (nnmg_level_set_rhs_split) are then timed and the faster kept.  Synchronizes the
 * device; hierarchies holding the level re-capture their V-cycle graphs.
 * nnmg_level_set_variant forces a variant for both precisions,
 * nnmg_level_set_variant_prec for one; nnmg_level_variant reads the variant
 * of one precision. */
int nnmg_level_tune(nnmg_level* level, nnmg_prec prec, int reps, nnmg_tune_result* res);
int nnmg_level_set_variant(nnmg_level* level, int variant);
int nnmg_level_set_variant_prec(nnmg_level* level, nnmg_prec prec, int variant);
int nnmg_level_variant(const nnmg_level* level, nnmg_prec prec, int* variant);
/* Several right-hand sides in one operator launch (the _multi calls and the
 * solves with several right-hand sides): split = 1 gives each right-hand side
 * its own row of workgroups, split = 0 lets every workgroup loop over them.
 * nnmg_level_tune times both on small levels (fewer than 16384 wavefronts
 * per launch) and keeps the faster.  Same results either way (each
 * right-hand side is summed in the same order). */
int nnmg_level_set_rhs_split(nnmg_level* level, nnmg_prec prec, int split);
/* Cells per workgroup of the operator kernels (the tile each workgroup
 * sweeps).  The level's data are laid out in blocks of `layout_cells` cells
 * (3D: 16, 7, 4, 5 for degree 1..4; 2D: 64 / (k+1)), one block per wavefront
 * (degree 4 in 3D: two); a workgroup takes one block or two consecutive ones,
 * `cells` = layout_cells or 2 layout_cells.  The two layout blocks of a
 * workgroup keep separate LDS regions and sum in the same order as alone, so
 * the results are bitwise the same either way.  Two blocks apply to the
 * Laplace contribution-slot variants; the atomic variants and the elasticity
 * operator take one (setting two there: NNMG_ERR_UNSUPPORTED for elasticity,
 * ignored by the atomic variants, which report layout_cells).
 * nnmg_level_tune times both for the variant it keeps and keeps the faster.
 * nnmg_level_cells_per_block also returns the number of layout blocks (with
 * two per workgroup, an odd count leaves the last workgroup half idle).
 * Other values of `cells`: NNMG_ERR_INVALID_ARG.  Synchronizes the device;
 * hierarchies holding the level re-capture their graphs. */
int nnmg_level_set_cells_per_block(nnmg_level* level, nnmg_prec prec, int cells);
int nnmg_level_cells_per_block(const nnmg_level* level, nnmg_prec prec, int* cells, int* layout_cells,
                               int64_t* layout_blocks);

/* Times the restriction (paper §2, eq. residual2) with 4 << v lanes per
 * coarse cell, v = 0..4, and keeps the fastest (same contract as
 * nnmg_level_tune).  The restriction of 3D cells of degree 3 and 4 takes one
 * wavefront per coarse cell and value whatever the team: there only v = 0 is
 * timed (n_variants = 1).  nnmg_transfer_set_team forces a team of 4, 8, 16, 32 or
 * 64 lanes; nnmg_transfer_team reads it. */
int nnmg_transfer_tune(nnmg_transfer* transfer, nnmg_prec prec, int reps, nnmg_tune_result* res);
int nnmg_transfer_set_team(nnmg_transfer* transfer, int team);
int nnmg_transfer_team(const nnmg_transfer* transfer, int* team);

/* ------------------------------------------------------------------------ */
/* Hierarchy, V-cycle and PCG (paper §2 Algorithm V_cycle; §4 recipe)          */
/* ------------------------------------------------------------------------ */

/* levels: n_levels handles, coarse -> fine; transfers: n_levels - 1 handles,
 * transfers[i] between levels[i+1] (fine) and levels[i] (coarse).  Estimates
 * the Chebyshev interval of every level above the coarsest (Jacobi-CG
 * Lanczos), and factorises the coarsest operator into a dense float64
 * inverse.  opts may be NULL.  Synchronous. */
int nnmg_hierarchy_create(nnmg_ctx* ctx, nnmg_level* const* levels, int n_levels,
                          nnmg_transfer* const* transfers, const nnmg_mg_opts* opts,
                          nnmg_hierarchy** out);
void nnmg_hierarchy_destroy(nnmg_hierarchy* hierarchy);

int nnmg_get_cheb_bounds(const nnmg_hierarchy* h, int level, double* lo, double* hi);
int nnmg_set_cheb_bounds(nnmg_hierarchy* h, int level, double lo, double hi);

/* z = V(r): one V-cycle on the finest level with a zero initial guess
 * (Algorithm V_cycle): Chebyshev-Jacobi pre-smoothing, residual, restriction,
 * recursion, exact float64 coarse solve (dense inverse of the unconstrained
 * block; in a float64 cycle plus one refinement step whose residual uses the
 * level's operator), prolongation, post-smoothing from the current iterate.
 * r and z are vectors of the finest level in `prec`.  Asynchronous. */
int nnmg_vcycle(nnmg_hierarchy* h, nnmg_prec prec, const void* r_dev, void* z_dev, void* stream);

/* nnmg_vcycle for nrhs interleaved right-hand sides (layout and limits as for
 * nnmg_vmult_multi): one V-cycle whose every launch carries all of them. */
int nnmg_vcycle_multi(nnmg_hierarchy* h, nnmg_prec prec, int nrhs, const void* r_dev, void* z_dev, void* stream);

/* Float64 CG from x0 = 0 preconditioned by one V-cycle in opts->vcycle_prec
 * (paper §4: V-cycle in single, CG in double precision).  b_dev and x_dev are
 * float64 vectors of the finest level.  Synchronous.  Returns NNMG_OK,
 * NNMG_ERR_NOT_CONVERGED or NNMG_ERR_BREAKDOWN (res->status says the same;
 * x_dev then holds the last iterate). */
int nnmg_pcg_solve(nnmg_hierarchy* h, const double* b_dev, double* x_dev, const nnmg_cg_opts* opts,
                   nnmg_cg_result* res, void* stream);

/* nrhs independent CG solves run in lockstep, one preconditioner V-cycle and
 * one operator product for all of them per iteration (b_dev, x_dev
 * interleaved as for nnmg_vmult_multi).  Each right-hand side keeps its own
 * scalars and stopping test; once it has converged (or broken down) it is
 * frozen, so its x and iteration count are those of nnmg_pcg_solve on it
 * alone, while the others go on.  res: host [nrhs]; opts->history, if set:
 * host [nrhs][max_it + 1].  Returns NNMG_ERR_BREAKDOWN if any right-hand side
 * broke down, else NNMG_ERR_NOT_CONVERGED if any did not converge, else
 * NNMG_OK.  Synchronous. */
int nnmg_pcg_solve_multi(nnmg_hierarchy* h, int nrhs, const double* b_dev, double* x_dev,
                         const nnmg_cg_opts* opts, nnmg_cg_result* res, void* stream);

/* Per-component times: when enabled, every V-cycle records HIP events around
 * its components.  nnmg_hierarchy_profile writes the accumulated milliseconds
 * ms[level][c] (host [n_levels][6], levels coarse -> fine; c = pre-smoother,
 * residual, restriction, coarse solve, prolongation, post-smoother) and
 * resets the accumulators; it synchronises the hierarchy's last stream. */
int nnmg_hierarchy_set_profiling(nnmg_hierarchy* h, int enabled);
int nnmg_hierarchy_profile(nnmg_hierarchy* h, double* ms);

/* Device memory a solve of nrhs right-hand sides needs beyond the
 * hierarchy's fixed data (work vectors of both precisions, CG vectors,
 * contribution and restriction buffers); the serving loop admits requests
 * by it. */
int nnmg_hierarchy_footprint(const nnmg_hierarchy* h, int nrhs, size_t* bytes);

/* ------------------------------------------------------------------------ */
/* Serving loop with continuous batching                                       */
/* ------------------------------------------------------------------------ */
/* A server owns one loop thread and max_active streams.  Requests name a
 * resident hierarchy and nrhs right-hand sides (the solve of
 * nnmg_pcg_solve_multi, paper §4 recipe).  The loop admits queued requests,
 * in the policy's order but without letting one that does not fit hold back
 * later ones, whenever a slot is free, the request's footprint fits the
 * memory budget beside the running ones (a request alone is always
 * admitted), a large request would not exceed max_large running large ones,
 * and its hierarchy serves no other request.  Running requests advance one CG
 * stage at a time on their own streams, so their kernels overlap on the
 * device.  Each request makes exactly the launches of nnmg_pcg_solve_multi:
 * its result is the same alone and in the mix.  A hierarchy must not be used
 * by other calls while a request on it runs. */
typedef struct nnmg_server nnmg_server;

typedef struct {
    int max_active;        /* requests running at once (default 4, 1..64) */
    size_t memory_budget;  /* bytes of footprint the running requests may hold together (default 64 GiB) */
    int policy;            /* admission order: NNMG_ADMIT_ARRIVAL (default) or NNMG_ADMIT_SMALLEST */
    double aging_ms;       /* NNMG_ADMIT_SMALLEST: a request queued this long is taken in arrival order,
                              before every younger one (default 250) */
    double large_work;     /* a request whose expected work (fine DoFs x nrhs) is at least this is large
                              (default 0: no request is large) */
    int max_large;         /* large requests running at once (default 64: no limit below max_active) */
} nnmg_server_opts;

/* Admission orders of the serving loop: arrival order, or smallest expected
 * work (fine DoFs x nrhs) first with the aging bound of nnmg_server_opts. */
enum { NNMG_ADMIT_ARRIVAL = 0, NNMG_ADMIT_SMALLEST = 1 };

typedef struct {
    double queued_ms;  /* submit -> admitted */
    double run_ms;     /* admitted -> finished */
    double total_ms;   /* submit -> finished */
} nnmg_request_times;

typedef struct {
    int64_t submitted, completed;
    int running, pending;    /* now */
    int max_running;         /* most requests running at once so far */
    size_t reserved;         /* footprint held by the running requests now */
    size_t max_reserved;     /* most footprint held at once so far */
} nnmg_server_stats;

void nnmg_default_server_opts(nnmg_server_opts* opts);
int nnmg_server_create(nnmg_ctx* ctx, const nnmg_server_opts* opts, nnmg_server** out);
/* Finishes every queued request, then stops the loop.  NULL is a no-op. */
void nnmg_server_destroy(nnmg_server* server);

/* Queues a request and returns at once with its ticket.  b_dev (float64
 * [n_dofs][nrhs], complete on the device: synchronize the stream that wrote
 * it first) and x_dev must stay valid, and b_dev unchanged, until
 * nnmg_server_wait returns; opts may be NULL (defaults), opts->history (host
 * [nrhs][max_it + 1]) likewise.  Errors: INVALID_ARG (arguments, nrhs out of
 * 1..8, server shutting down). */
int nnmg_server_submit(nnmg_server* server, nnmg_hierarchy* h, int nrhs, const double* b_dev, double* x_dev,
                       const nnmg_cg_opts* opts, int64_t* ticket);
/* nnmg_server_submit for a set of n_replicas equivalent hierarchies (built
 * over the same levels and transfers with the same options, so any of them
 * gives the same result): the request runs on whichever is idle first.  A hot
 * mesh can so serve several requests at a time, each replica holding its own
 * work buffers (nnmg_hierarchy_footprint) beside the shared levels and
 * transfers. */
int nnmg_server_submit_any(nnmg_server* server, nnmg_hierarchy* const* replicas, int n_replicas, int nrhs,
                           const double* b_dev, double* x_dev, const nnmg_cg_opts* opts, int64_t* ticket);
/* *done = 1 once the request has finished. */
int nnmg_server_poll(nnmg_server* server, int64_t ticket, int* done);
/* Blocks until the request has finished, writes res (host [nrhs]) and times
 * (may be NULL), and retires the ticket.  Returns the request's status, as
 * nnmg_pcg_solve_multi would. */
int nnmg_server_wait(nnmg_server* server, int64_t ticket, nnmg_cg_result* res, nnmg_request_times* times);
int nnmg_server_get_stats(nnmg_server* server, nnmg_server_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* NNMG_H */
