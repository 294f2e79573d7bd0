/*
 * gofd.h -- C ABI of the grid-overlay finite difference (GoFD) library for the
 * fractional Laplacian on one AMD Instinct MI355X (gfx950).
 *
 * Method: W. Huang and J. Shen, "A grid-overlay finite difference method for
 * the fractional Laplacian on arbitrary bounded domains".  The library
 * discretises the homogeneous Dirichlet problem (-Delta)^s u = f in Omega,
 * u = 0 outside Omega, 0 < s < 1 (eq. FL-1), on an unstructured simplicial
 * mesh T_h overlaid by a uniform grid T_FD, through
 *
 *     A_h = D_h^{-1} (I_h^FD)^T A_FD I_h^FD                      (eq. Ah-1)
 *
 * where I_h^FD is P1 interpolation from the mesh to the grid (eq. IhFD-1),
 * D_h holds its column sums, and A_FD is the multilevel Toeplitz matrix of the
 * uniform-grid FD approximation (eqs. T-1, A-1, AFD-1), applied through a
 * zero-padded circulant embedding and FFTs (eq. AU-1).  The linear system is
 * GoFD-2 on the interior vertices,
 *
 *     (I^T A_FD I) u = h^{2s} I^T f_FD                            (eq. GoFD-2)
 *
 * solved by preconditioned conjugate gradients with the incomplete Cholesky
 * factor (level-1 fill) of A_h^(p) = I^T A_FD^(p) I (eq. Ah-4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: GOFD_OK (0) on success, a negative gofd_status otherwise;
 *    gofd_last_error(ctx) gives a human-readable reason.  On error no output
 *    buffer is guaranteed to hold anything meaningful.
 *  - Pointers named *_dev are device pointers (HIP global memory of the
 *    context's device), owned by the caller, read-only unless documented as an
 *    output, and must stay valid until the work enqueued by the call has
 *    finished on the context's stream.  Pointers without the suffix are host
 *    pointers.
 *  - Work is enqueued on the context's stream.  Calls that return results on
 *    the host (info structs, T tables) synchronise that stream before
 *    returning; gofd_apply_* calls are asynchronous.
 *  - Handles (gofd_transfer, gofd_fdop, gofd_precond) are owned by the library
 *    and freed with their *_free function; a handle copies whatever it needs
 *    from the inputs, so inputs may be freed after the creating call returns.
 *  - Grid geometry: the cube (c - R, c + R)^d carries W = 2N+1 nodes per axis
 *    with spacing h = R/N (Section 3.1).  Node i along axis a is located at
 *    (c_a - R) + i*h with each operation rounded separately in double
 *    precision (no fused multiply-add).  Grid arrays are stored in C order with
 *    the x index fastest: node (i_0, .., i_{d-1}) has linear number
 *    i_0 + W i_1 (+ W^2 i_2), the natural ordering.
 *  - Vertex vectors have length N_v in the mesh's vertex numbering.  With
 *    nrhs > 1, right-hand sides / fields are stored one after another.
 */
#ifndef GOFD_H
#define GOFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GOFD_OK = 0,
  GOFD_E_ARG = -1,            /* bad pointer, size, dimension, s not in (0,1), N < 1 ... */
  GOFD_E_DEGENERATE = -2,     /* a mesh element has zero volume                          */
  GOFD_E_RANK = -3,           /* (2N+1)^d < N_v: I cannot have full column rank          */
  GOFD_E_ZERO_COLSUM = -4,    /* an interior vertex has D_j = 0 (grid too coarse)         */
  GOFD_E_NOT_CONVERGED = -5,  /* iteration limit reached before the tolerance             */
  GOFD_E_BREAKDOWN = -6,      /* CG breakdown (p^T K p <= 0) or a non-finite value        */
  GOFD_E_HIP = -7,            /* a HIP runtime call failed                                */
  GOFD_E_OOM = -8,            /* device or host allocation failed                         */
  GOFD_E_NUMERIC = -9,        /* exact-arithmetic capacity exceeded in point location     */
  GOFD_E_UNSUPPORTED = -10    /* valid request this build does not implement              */
} gofd_status;

typedef struct gofd_ctx_s* gofd_ctx;
typedef struct gofd_transfer_s* gofd_transfer;
typedef struct gofd_fdop_s* gofd_fdop;
typedef struct gofd_precond_s* gofd_precond;

/* Overlay grid T_FD (Section 3.1): W = 2N+1 nodes per axis, h = R/N. */
typedef struct {
  int d;              /* 2 or 3                                          */
  int N;              /* half the number of intervals per axis, N >= 1   */
  double R;           /* half side of the cube                           */
  double center[3];   /* cube centre (unused entries ignored)            */
} gofd_grid;

/* ---------------------------------------------------------------- context */

/* Create a context bound to the current HIP device and the given stream
 * (a hipStream_t passed as void*; NULL means the null stream).
 * Errors: GOFD_E_ARG (out == NULL), GOFD_E_HIP, GOFD_E_OOM. */
int gofd_create(gofd_ctx* out, void* hip_stream);
/* Destroy a context (handles created from it must be freed first). */
int gofd_destroy(gofd_ctx ctx);
/* Re-bind the context to another stream of the same device. */
int gofd_set_stream(gofd_ctx ctx, void* hip_stream);
/* Last error message of this context (static storage owned by ctx). */
const char* gofd_last_error(gofd_ctx ctx);
/* Name of a status code. */
const char* gofd_strerror(int status);

/* ---------------------------------------------------------------- transfer */

typedef struct {
  int64_t n_nodes;          /* W^d                                                        */
  int64_t n_inside;         /* grid nodes lying in a closed mesh element                  */
  int64_t nnz;              /* structural nonzeros of I: (d+1) * n_inside                 */
  int64_t n_interior;       /* vertices not on a boundary facet                           */
  int64_t n_boundary;       /* Dirichlet vertices (on a facet owned by one element)       */
  double dmin_interior;     /* min D_j over interior vertices                             */
  double a_h;               /* minimum element height                                     */
  double h_bound;           /* a_h / ((d+1) sqrt(d)), the sufficient spacing of eq. hFD-1  */
  int64_t exact_tests;      /* orientation signs decided by exact expansion arithmetic    */
  int64_t max_col_count;    /* largest number of grid nodes touching one vertex          */
  int64_t rp_slots;         /* 2D: partial sums of the row-pair form of I^T used inside   */
                            /* CG (one per vertex and row pair it touches); 0 if absent  */
  int64_t rp_entries;       /* 2D: stored entries of that form (with per-thread padding)  */
  int64_t rp_seg_rows;      /* 2D: 1 if the per-node segment rows of the FP32 gather      */
                            /* through the row-pair slots were built, else 0              */
  double kernel_us[8];      /* device time of the build's stages (GOFD_TR_K_*), from HIP  */
                            /* events at each kernel's start and end (the scan: around it) */
} gofd_transfer_info;

/* Stages of gofd_build_transfer timed in gofd_transfer_info.kernel_us. */
enum {
  GOFD_TR_K_RECORDS = 0,  /* per element: vertex 0 and the barycentric gradients              */
  GOFD_TR_K_LOCATE = 1,   /* point location: each element's bounding box, exact orientation  */
  GOFD_TR_K_COUNT = 2,    /* entries per vertex                                                */
  GOFD_TR_K_SCAN = 3,     /* column offsets (exclusive scan)                                   */
  GOFD_TR_K_FILL = 4,     /* barycentric weights into the vertex-major structure               */
  GOFD_TR_K_SORT = 5,     /* each vertex's entries in ascending node order                     */
  GOFD_TR_K_ROWS = 6,     /* node-major rows of the gather (2D FP32 rows, 3D rows)             */
  GOFD_TR_K_COLSUM = 7    /* column sums D and the scalings                                    */
};

/* Build I_h^FD, its transpose structure and D_h (Section 3.1, eqs. interp-1 to
 * IhFD-1; D_h after eq. Ah-1 and Lemma IhFD-1(iv)).
 *   X_dev      N_v x d doubles, row-major vertex coordinates.
 *   elems_dev  N_e x (d+1) int32, 0-based vertex ids, either orientation.
 *   grid       overlay grid (host struct).
 * Point location: node k belongs to the element with the smallest id among
 * the closed elements that contain it (exact orientation signs); a node in no
 * closed element has a zero row.  The barycentric weights of node k are
 * lambda = E^{-1}[x_k; 1] (proof of the simplex interpolation lemma).
 * Dirichlet vertices are the vertices of facets owned by a single element;
 * the solve keeps them at zero (remark after eq. GoFD-2).
 * info (host, nullable) receives the statistics above.
 * Errors: GOFD_E_ARG, GOFD_E_DEGENERATE, GOFD_E_RANK, GOFD_E_ZERO_COLSUM,
 * GOFD_E_NUMERIC, GOFD_E_HIP, GOFD_E_OOM. */
int gofd_build_transfer(gofd_ctx ctx, int d, int64_t nv, const double* X_dev, int64_t ne,
                        const int32_t* elems_dev, const gofd_grid* grid, gofd_transfer* out,
                        gofd_transfer_info* info);
int gofd_transfer_free(gofd_transfer tr);

/* Copy parts of a transfer to caller buffers (device pointers, enqueued on the
 * stream).  Sizes: ELEM int32[W^d] (element of each node or -1);
 * ELL_VERTS int32[W^d*(d+1)] and ELL_WEIGHTS double[W^d*(d+1)] (vertex ids and
 * barycentric weights of each node's element, zero rows for outside nodes,
 * vertex ids -1 there); CSC_OFFSETS int32[N_v+1]; CSC_NODES int32[nnz] (grid
 * node of each entry, vertex-major, ascending node number inside a vertex);
 * CSC_WEIGHTS double[nnz]; D double[N_v]; BOUNDARY uint8[N_v] (1 = Dirichlet). */
typedef enum {
  GOFD_TR_ELEM = 0,
  GOFD_TR_ELL_VERTS = 1,
  GOFD_TR_ELL_WEIGHTS = 2,
  GOFD_TR_CSC_OFFSETS = 3,
  GOFD_TR_CSC_NODES = 4,
  GOFD_TR_CSC_WEIGHTS = 5,
  GOFD_TR_D = 6,
  GOFD_TR_BOUNDARY = 7
} gofd_transfer_part;
int gofd_transfer_export(gofd_ctx ctx, gofd_transfer tr, int part, void* dst_dev);

/* ---------------------------------------------------------------- FD operator */

typedef struct {
  int64_t M;        /* finest quadrature level M (power of two); 0 = the paper's
                       default: 2^14 for d = 2, 2^11 for d = 3, raised if needed so
                       that M/2 >= 2(2N)+1                                          */
  int richardson;   /* 1 = combine levels M and M/2 (the paper), 0 = level M only  */
} gofd_fdw_opts;

/* Toeplitz coefficients T_p, p in {0..2N}^d, of the FD fractional Laplacian
 * (eqs. T-0, T-1) by Filon's rule with piecewise-linear psi~ (eq. Tp-1D-2,
 * applied along every axis) and Richardson extrapolation over M and M/2
 * (Section 2.3), computed on the device; then the real, even DFT of the
 * circulant embedding used by the FFT product (eq. AU-1).  h^{2s} is stored
 * for the right-hand side of eq. GoFD-2.  opts may be NULL (defaults).
 * Errors: GOFD_E_ARG (s not in (0,1), bad grid), GOFD_E_HIP, GOFD_E_OOM. */
int gofd_fd_weights(gofd_ctx ctx, double s, const gofd_grid* grid, const gofd_fdw_opts* opts,
                    gofd_fdop* out);

/* Same operator from a caller-supplied T octant (host, (2N+1)^d doubles in the
 * grid-array layout: T[p_0 + W p_1 (+ W^2 p_2)] = T_{p}).  s only scales the
 * right-hand side (h^{2s}). */
int gofd_fdop_from_table(gofd_ctx ctx, double s, const gofd_grid* grid, const double* T_host,
                         gofd_fdop* out);
/* Copy the T octant ((2N+1)^d doubles) to a host buffer (synchronises). */
int gofd_fdop_get_table(gofd_ctx ctx, gofd_fdop op, double* T_host);
int gofd_fdop_free(gofd_fdop op);

/* Flags of the apply calls. */
enum {
  GOFD_FP32_GRID = 1,     /* grid-side arrays and FFTs in single precision (mesh vectors,
                             weights and the final accumulation stay double)             */
  GOFD_SYMMETRIC = 2,     /* apply A~_h = D^{-1/2} I^T A_FD I D^{-1/2} (eq. Ah-3)           */
  GOFD_UNSCALED = 4,      /* apply I^T A_FD I (the matrix of eq. GoFD-2, all vertices)     */
  GOFD_SCALE_H2S = 8,     /* multiply the result by h^{-2s} (the operator of eq. GoFD-1)   */
  GOFD_INTERIOR = 16      /* zero the input and output on Dirichlet vertices              */
};

/* y = A_FD v on the grid (eq. AFD-1) for nrhs fields of W^d doubles.
 * v_dev and y_dev may not alias. */
int gofd_apply_afd(gofd_ctx ctx, gofd_fdop op, int nrhs, const double* v_dev, double* y_dev,
                   int flags);

/* y = A_h u = D^{-1} I^T A_FD I u (eq. Ah-1) for nrhs vertex vectors of N_v
 * doubles; variants by flags as above.  u_dev and y_dev may not alias.
 * Errors: GOFD_E_ARG (grids of op and tr differ, nrhs < 1), GOFD_E_HIP. */
int gofd_apply_Ah(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int nrhs, const double* u_dev,
                  double* y_dev, int flags);

/* Allocation-free variant of gofd_apply_Ah, for callers that cannot allocate
 * device memory while they run: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, flags, results and
 * errors as gofd_apply_Ah (the operator must have been created in ctx).  The
 * product's grid workspaces (the grid result A_FD I u, the gathered field I u
 * and the spectra of the FFT passes) live in one static device array of
 * GOFD_NOALLOC_WS_BYTES bytes per GPU, which the library holds from its load
 * until the process ends, instead of buffers of the operator; the call
 * allocates nothing.  It needs, with b = 8 (b = 4 with GOFD_FP32_GRID) and
 * each part rounded up to 256 bytes,
 *   2 b W^d nrhs + 2 b W (L/2) nrhs                        (d = 2),
 *   2 b W^3 nrhs + 2 b 4 ceil((L/2+1)/4) W (W + L) nrhs    (d = 3),
 * where L is the FFT period (4N rounded up to a power of two); a request
 * beyond the array fails with GOFD_E_ARG and a message giving the bytes
 * needed (2D double precision: one field at W = 1025, seven at W = 513).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, threads or contexts)
 * race, and the caller must order them.  Enqueued on the context's stream;
 * asynchronous.  GOFD_E_HIP if the runtime could not give the array's device
 * address when the context was created. */
enum { GOFD_NOALLOC_WS_BYTES = 64 << 20 };
int gofd_apply_Ah_noalloc(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int nrhs, const double* u_dev,
                          double* y_dev, int flags);

/* Schedules of the FFT passes, properties of the context that apply to every
 * later product of the same (FFT period L, precision); results agree between
 * schedules to rounding.
 *  - 2D column pass (transform the spectrum columns, multiply by the kernel's
 *    spectrum, transform back; eq. AU-1): GOFD_N_COL_SCHED schedules (values
 *    per thread and column slots per block: 0 = 16/2, the built-in default,
 *    1 = 16/1, 2 = 8/2, 3 = 16/4).
 *  - 2D first row pass of the products from a grid field (apply calls, FP64
 *    CG, residual replacements): 8 or 16 values per thread where both are
 *    built (L >= 1024; 0 = the default, 8).  The FP32 CG's row pass, which
 *    gathers through the row-pair slots, keeps 16.
 *  - 3D y/z/y passes: schedule 0 (four column slots per block where they fit,
 *    the default) or 1 (two).
 * gofd_autotune times the schedules for the given grid's period on the device
 * (zero fields of the grid's window, each timed over repeated launches after
 * untimed ones; GOFD_FP32_GRID in flags selects the precision), installs the
 * fastest (the default unless another is at least 5 % faster) and reports:
 * sched (host, nullable) receives 2 ints, the column schedule (3D: the y/z/y
 * schedule) and the row pass's values per thread (0 if not tuned);
 * times (host, nullable) receives GOFD_N_TUNE_TIMES average durations in ms:
 * 2D: times[0..3] the column schedules, times[4..5] the row pass at 8 and 16;
 * 3D: times[0..1]; entries not timed are +inf.  Synchronises.
 * gofd_set_schedule installs a known schedule (e.g. from a cache of earlier
 * tuning runs): the column schedule, or with GOFD_SCHED_ROWS in flags the row
 * pass's values per thread (0, 8, 16), or in 3D the y/z/y schedule (0, 1).
 * Errors: GOFD_E_ARG (bad grid or schedule number), GOFD_E_OOM, GOFD_E_HIP. */
enum { GOFD_N_COL_SCHED = 4, GOFD_N_TUNE_TIMES = 6, GOFD_SCHED_ROWS = 256 };
int gofd_autotune(gofd_ctx ctx, const gofd_grid* grid, int flags, int* sched, double* times);
int gofd_set_schedule(gofd_ctx ctx, const gofd_grid* grid, int flags, int sched);

/* Timing of one kernel of the K product in isolation (for roofline reports):
 * launches kernel `which` (GOFD_K_PASS_A: first FFT pass (rows), PASS_B: the
 * column pass with the spectral multiply, PASS_C: last FFT pass, SCATTER: the
 * I^T reduction, GATHER: the interpolation I u onto the grid) `reps` times on the library's stream between two HIP events,
 * after one untimed launch, with nrhs fields taken from u_dev (N_v doubles
 * each), and writes the average duration in milliseconds to *avg_ms (host).
 * Synchronises.  Errors: GOFD_E_ARG, GOFD_E_HIP. */
enum { GOFD_K_PASS_A = 0, GOFD_K_PASS_B = 1, GOFD_K_PASS_C = 2, GOFD_K_SCATTER = 3, GOFD_K_GATHER = 4 };
int gofd_time_kernel(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int which, int nrhs, const double* u_dev,
                     int flags, int reps, double* avg_ms);

/* ---------------------------------------------------------------- solve */

typedef enum {
  GOFD_PC_NONE = 0,       /* plain CG                                                      */
  GOFD_PC_DIAG = 1,       /* M = D_h: CG on the symmetric form A~_h (eq. Ah-3)             */
  GOFD_PC_IC1_5 = 5,      /* IC(1) of I^T A_FD^(5) I  (Section 3.3, 2D)                     */
  GOFD_PC_IC1_9 = 9,      /* IC(1) of I^T A_FD^(9) I  (Section 3.3, 2D)                     */
  GOFD_PC_IC1_27 = 27,    /* IC(1) of I^T A_FD^(27) I (Example 4, 3D)                       */
  GOFD_PC_MULTICOLOR = 256, /* flag added to an IC kind: the factor in multicolour order      */
  GOFD_PC_LAPLACIAN = 512,  /* flag added to an IC kind: the discrete Laplacian on the kind's
                               pattern in place of A_FD's entries (Section 3.3)              */
  GOFD_PC_BLOCK_MULTICOLOR = 1024 /* flag added to an IC kind: the factor in block multicolour
                               order (exclusive with GOFD_PC_MULTICOLOR)                     */
} gofd_pc_kind;

typedef struct {
  double shift;           /* alpha of the final factor of A + alpha diag(A) (0 = none)    */
  int64_t nnz_L;          /* nonzeros of the lower factor                                  */
  int levels;             /* dependency levels of the forward triangular solve             */
  double setup_ms;        /* host + device setup time                                      */
  int colours;            /* GOFD_PC_MULTICOLOR: colours of the ordering (0 otherwise)     */
  int64_t apply_bytes;    /* GOFD_PC_BLOCK_MULTICOLOR: algorithmic bytes of one application
                             (both triangular solves, one right-hand side): each entry to
                             another block (FP32 value, int32 column) and each FP32 16 x 16
                             block inverse read once per solve, block starts and slab
                             offsets, the permutation twice, and the vectors: r read, y
                             written and read twice, the upper solve's output written and
                             read once, u written (8 bytes per vertex each); 0 otherwise */
} gofd_precond_info;

/* Build a preconditioner for eq. GoFD-2 on the interior block.  For the IC(1)
 * kinds: the entries of A_FD on the 5/9/27-point pattern (Section 3.3), the
 * sparse triple product I^T A_FD^(p) I, a level-of-fill <= 1 incomplete
 * Cholesky factorisation in the mesh's vertex order (pivot <= 0: restart on
 * A + alpha diag(A), alpha = 1e-3 doubling), uploaded with its dependency
 * levels for the triangular solves.  With GOFD_PC_MULTICOLOR added to the
 * kind, the vertices are first coloured greedily (in vertex order, each the
 * smallest colour none of its neighbours in A^(p) has) and ordered by
 * (colour, vertex); the factor is that of P A P^T with level-1 fill kept only
 * between vertices of different colours, so a colour's rows depend only on
 * rows of other colours: each colour is one device-wide launch per triangular
 * solve (GOFD_E_UNSUPPORTED above 64 colours).  With GOFD_PC_LAPLACIAN added,
 * the matrix factored is I^T (-Delta_h) I with the discrete Laplacian on the
 * kind's pattern (up to a factor: p - 1 at the centre, -1 at the other p - 1
 * points; the standard 5-point one and the isotropic 9- and 27-point ones), the
 * Laplacian taking the place of A_FD in the stiffness matrix as Section 3.3
 * allows; it does not depend on s.  With GOFD_PC_BLOCK_MULTICOLOR added: the
 * vertices are grouped into blocks of at most 16 (in vertex order, a vertex
 * not yet placed starts a block that takes unplaced vertices breadth first,
 * neighbours in A^(p) in increasing order), the graph of the blocks is
 * coloured in smallest-last order (least degree removed first, ties to the
 * smaller block; coloured in reverse removal order, each block the smallest
 * free colour), the vertices are ordered by (block
 * colour, block, vertex), and the level-1 fill is kept inside a block and
 * between different colours: one device-wide launch per colour and solve,
 * each block's own rows solved within one wavefront; colours reports the
 * block colours.  Setup runs on the host (the
 * factor is sequential by nature); applies run on the device.  info nullable. */
int gofd_precond_create(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int kind, gofd_precond* out,
                        gofd_precond_info* info);
int gofd_precond_free(gofd_precond pc);
/* Export the IC factor L (lower CSR over all N_v vertices; Dirichlet rows are
 * identity rows).  Sizes from info->nnz_L; host buffers (synchronises). */
int gofd_precond_export(gofd_ctx ctx, gofd_precond pc, int32_t* rowptr_host, int32_t* cols_host,
                        double* vals_host);
/* Elimination order of the factor: row i of L is vertex perm_host[i] (N_v
 * int32, host; the identity without GOFD_PC_MULTICOLOR).  The factor exported
 * above is in that order. */
int gofd_precond_export_order(gofd_ctx ctx, gofd_precond pc, int32_t* perm_host);

enum { GOFD_F_GRID = 0, GOFD_F_VERTEX = 1 };
enum {
  GOFD_MODE_FP64 = 0,            /* every product in double precision                         */
  GOFD_MODE_FP32_REFINE = 1,     /* FP32-grid CG corrections inside FP64 iterative refinement */
  GOFD_MODE_FP32_RELIABLE = 2    /* one CG run with FP32-grid products whose residual is      */
                                 /* replaced by the FP64 true residual b - K x whenever it    */
                                 /* has dropped by the factor inner_tol since the last        */
                                 /* replacement, and before stopping (reliable updating,      */
                                 /* Sleijpen and van der Vorst 1996)                          */
};

typedef struct {
  int mode;              /* GOFD_MODE_*                                                     */
  int max_iter;          /* total CG iterations allowed (0 = 20000)                         */
  int check_every;       /* host reads of the CG state every k iterations (0 = 8); without  */
                         /* a graph the chunks shrink to 2 iterations near the tolerance    */
  double inner_tol;      /* FP32_REFINE: relative tolerance of each correction solve (0 =   */
                         /* 1e-5); FP32_RELIABLE: residual drop between replacements (0 = 1e-2) */
  int max_refine;        /* FP32 mode: maximum outer refinement steps (0 = 30)              */
  int use_graph;         /* 1: capture k CG iterations in a hipGraph and replay it; 0: launch */
                         /* the kernels directly (the default: shorter gaps on gfx950)      */
  double* history;       /* optional host array of max_iter+1 relative residuals, or NULL   */
  double* stage_ms;      /* optional host array of GOFD_N_STAGES: the iterations then run   */
                         /* without a graph, each stage bracketed by HIP events on the       */
                         /* library's stream, and the average milliseconds per launch of     */
                         /* every stage are written here (0 for a stage that never ran)      */
  const double* x0;      /* gofd_solve only: optional device array of nrhs * N_v doubles,    */
                         /* the initial guess (Dirichlet entries ignored; NULL = 0).  CG    */
                         /* then runs on the correction K d = b - K x0 with the stop still  */
                         /* ||b - K u|| <= tol ||b||, and u = x0 + d                         */
} gofd_solve_opts;

/* stages of one CG iteration, in the order of stage_ms */
enum { GOFD_ST_GATHER = 0, GOFD_ST_PASS_A = 1, GOFD_ST_PASS_B = 2, GOFD_ST_PASS_C = 3, GOFD_ST_SCATTER = 4,
       GOFD_ST_PRECOND = 5, GOFD_N_STAGES = 6 };

typedef struct {
  int iterations;        /* CG iterations (all refinement steps)                            */
  int refinements;       /* FP64 residual recomputations (FP32 modes)                       */
  double rel_residual;   /* ||b - K u|| / ||b|| recomputed in FP64 at exit                  */
  double time_ms;        /* wall time of the call                                           */
  int status;            /* GOFD_OK or the error returned                                   */
} gofd_solve_info;

/* Solve eq. GoFD-2 (f on the grid, f_loc = GOFD_F_GRID: W^d doubles per rhs,
 * values outside the mesh are ignored since their rows of I are zero) or
 * eq. GoFD-3 (f_loc = GOFD_F_VERTEX: N_v doubles per rhs) for u on the
 * vertices, with u = 0 on Dirichlet vertices, to ||b - K u||_2 <= tol ||b||_2
 * (CG from u = 0, or from opts->x0).  pc may be NULL (plain CG) or a gofd_precond.
 *   f_dev: nrhs right-hand sides; u_dev: nrhs * N_v doubles (output).
 *   info: host array of nrhs entries (nullable).
 * Errors: GOFD_E_ARG, GOFD_E_NOT_CONVERGED, GOFD_E_BREAKDOWN, GOFD_E_HIP. */
int gofd_solve(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, gofd_precond pc, int nrhs,
               const double* f_dev, int f_loc, double tol, const gofd_solve_opts* opts,
               double* u_dev, gofd_solve_info* info);

/* Many independent problems (mesh, grid, s, right-hand sides) in one call:
 * problem q uses tr[q], op[q], pc[q] (nullable) and nrhs[q] right-hand sides
 * f_dev[q] -> u_dev[q].  Problems are grouped by grid shape (d, 2N+1 and the
 * FFT length); within a group the CG iterations of all (problem, rhs) items
 * advance together, every stage of an iteration one kernel launch for the
 * whole group (items index per-item descriptors of their mesh, vectors and
 * kernel spectrum), launched directly or from a hipGraph (opts->use_graph);
 * converged items are masked and, once few remain, the launches narrowed to
 * them.  IC(1) triangular solves: the block multicolour factors of a group's
 * problems in one launch per colour and direction, other orders per problem.
 * Groups run concurrently (a host thread and streams each, after the
 * context's stream on entry and before it on exit); one after another when
 * stage timing or a residual history is requested.
 * info: host array of sum(nrhs) entries in problem order (nullable).
 * Errors: as gofd_solve. */
int gofd_solve_batched(gofd_ctx ctx, int nprob, const gofd_transfer* tr, const gofd_fdop* op,
                       const gofd_precond* pc, const int* nrhs, const double* const* f_dev,
                       int f_loc, double tol, const gofd_solve_opts* opts, double* const* u_dev,
                       gofd_solve_info* info);

/* Gradients of a scalar loss L(u) of the GoFD-2 solution u (f on the grid)
 * by the adjoint method: lambda = K^{-1} dL/du (K is symmetric, same solver),
 * dL/df_FD = h^{2s} I lambda, dL/dI_kj = lambda_j r_k - (A_FD I lambda)_k u_j
 * with r = h^{2s} f_FD - A_FD I u, chained to the vertex coordinates through
 * d lambda_r/d X_{i,a} = -(E^{-1})_{r,a} lambda_i (point location held fixed).
 *   dLdu_dev, u_dev: N_v doubles (u from gofd_solve); f_dev: W^d doubles.
 *   grad_f_dev: W^d doubles or NULL; grad_X_dev: N_v*d doubles or NULL.
 *   lambda_dev: optional output of the adjoint solution (N_v doubles) or NULL. */
int gofd_solve_adjoint(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, gofd_precond pc,
                       const double* dLdu_dev, const double* u_dev, const double* f_dev, double tol,
                       const gofd_solve_opts* opts, double* grad_f_dev, double* grad_X_dev,
                       double* lambda_dev, gofd_solve_info* info);

/* ---------------------------------------------------------------- truncated CG */

typedef struct gofd_cg_tape_s* gofd_cg_tape;

typedef struct {
  int iterations;        /* n: CG iterations run                                           */
  int checkpoints;       /* stored checkpoints (iterations 0, c, 2c, ... <= n)             */
  double rel_residual;   /* sqrt(gamma_n / (b, b)) of the recursive residual               */
  int converged;         /* 1 if the tolerance stopped the iteration before max_iter       */
} gofd_cg_tape_info;

/* Conjugate gradients on eq. GoFD-2 (Section 3.2; f on the grid, W^d doubles,
 * one right-hand side), textbook form in double precision, started from
 * x0_dev (N_v doubles, Dirichlet entries ignored; NULL = 0) and stopped after
 * max_iter iterations or once ||r|| <= tol ||b|| (tol = 0: exactly max_iter
 * iterations unless the residual vanishes).  Writes x_n to x_dev (N_v).
 * The iterate (x, r, p) is kept on the device every ckpt_every = c
 * iterations (checkpoints 0, c, 2c, ...), with every iteration's gamma,
 * delta, alpha and beta, in the tape returned in *tape (library-owned, freed
 * with gofd_cg_tape_free; it refers to tr and op, which must outlive it).
 * Device memory of the tape: 3 N_v (max_iter / c + 1) + 4 (max_iter + 1)
 * doubles + a copy of f.  info (host, nullable).
 * Errors: GOFD_E_ARG, GOFD_E_BREAKDOWN (p^T K p <= 0 or non-finite: no tape),
 * GOFD_E_HIP, GOFD_E_OOM. */
int gofd_cg_checkpointed(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, const double* f_dev,
                         const double* x0_dev, int max_iter, double tol, int ckpt_every, double* x_dev,
                         gofd_cg_tape* tape, gofd_cg_tape_info* info);

/* Reverse-mode (unrolled) gradient of the truncated solve recorded in tape:
 * given xbar_dev = dL/dx_n (N_v doubles; Dirichlet entries ignored), the
 * gradients of L through the n CG iterations with respect to f (grad_f_dev,
 * W^d doubles), the vertex coordinates (grad_X_dev, N_v x d, with point
 * location held fixed) and x_0 (grad_x0_dev, N_v); each output nullable.
 * The iteration count n is held fixed (the stopping test is piecewise
 * constant).  The iterates of each segment of c iterations are recomputed
 * from its checkpoint, so the call costs about 2n + 2 products and holds c
 * vertex vectors (and c grid fields when grad_X_dev is given).  When the
 * truncated solve has converged the result approaches the adjoint of the
 * converged system (gofd_solve_adjoint).  Synchronises.
 * Errors: GOFD_E_ARG (tape from another context), GOFD_E_HIP, GOFD_E_OOM. */
int gofd_cg_unrolled_grad(gofd_ctx ctx, gofd_cg_tape tape, const double* xbar_dev, double* grad_f_dev,
                          double* grad_X_dev, double* grad_x0_dev);

/* Copy checkpoint j (0 <= j <= n / c) of a tape: x_{jc}, r_{jc}, p_{jc} to
 * device buffers of N_v doubles (each nullable), and the scalar record to a
 * host array of 4 (max_iter + 1) doubles (nullable): gamma_0..gamma_n, then
 * delta_i, alpha_i, beta_i for i < n, each array max_iter + 1 long.
 * Synchronises. */
int gofd_cg_tape_read(gofd_ctx ctx, gofd_cg_tape tape, int j, double* x_dev, double* r_dev, double* p_dev,
                      double* scalars_host);
int gofd_cg_tape_free(gofd_cg_tape tape);

/* ---------------------------------------------------------------- mesh adaptation (MMPDE), 2D */

/* Algorithm amGoFD of Section 4 moves the vertices of the triangulation
 * towards a mesh equidistributed in the metric of eq. MK-1 built from the
 * recovered Hessian of the current solution, by the moving mesh equations
 * (eqs. x-1, mmpde-1) applied to the energy of eq. I-h; the connectivity
 * never changes.  The GoFD solve on each new mesh goes through
 * gofd_build_transfer / gofd_solve as for any other mesh.
 *
 * Layout: X (N_v x 2 doubles, row-major), u (N_v doubles), elements
 * (N_e x 3 int32, vertex indices, counter-clockwise), vertex metrics Mv
 * (N_v x 3 doubles: m11, m12, m22 of the symmetric 2 x 2 tensor), element
 * metrics M_K (N_e x 3, same order), vertex Hessians (N_v x 3, same order).
 * All on the device.
 * The metric is a field of position: the piecewise-linear interpolant of
 * the vertex metrics on a background mesh Xb (for a move, the mesh it
 * starts from).  M_K is its value at the current centroid of K, located in
 * the background mesh by a walk across the edge opposite the most negative
 * barycentric coordinate (at most 4096 moves; beyond a boundary edge the
 * value is extrapolated from that edge's element).
 * Boundary vertices are those on an edge owned by one element.  With
 * GOFD_MMPDE_BOUNDARY_CIRCLE they slide along the unit circle (the normal
 * component of their velocity is removed and each step puts them back on
 * it), with GOFD_MMPDE_BOUNDARY_FIXED they stay where they are.
 * Sums over the elements around a vertex run in element order, and every
 * reduction in a fixed order, so every result is reproducible bit for bit.
 * Calls on one handle must not overlap. */
typedef struct gofd_mmpde_s* gofd_mmpde;

enum { GOFD_MMPDE_BOUNDARY_CIRCLE = 0, GOFD_MMPDE_BOUNDARY_FIXED = 1 };

/* Kernels of a move, for gofd_mmpde_kernel_stats. */
enum {
  GOFD_MMPDE_K_HESS = 0,      /* element Hessians by differences (once per step)                   */
  GOFD_MMPDE_K_FIELD = 1,     /* metric at the centroids (walks; once per trial)                     */
  GOFD_MMPDE_K_ENERGY = 2,    /* energy partials and inversion test (once per trial)                 */
  GOFD_MMPDE_K_CG_ELEM = 3,   /* CG: convergence test, beta, element Hessians times the new direction */
  GOFD_MMPDE_K_CG_VERT = 4,   /* CG: new direction stored, vertex sums, shift, projection, (p, w)     */
  GOFD_MMPDE_K_CG_UPDATE = 5, /* CG: alpha, x, r, preconditioner, partials                           */
  GOFD_MMPDE_N_KERNELS = 6
};

typedef struct {
  double avg_us[GOFD_MMPDE_N_KERNELS];    /* mean duration of the first (up to 32) launches, from HIP
                                             events recorded at each launch's start and end           */
  int64_t launches[GOFD_MMPDE_N_KERNELS]; /* launches of the move (CG kernels launched past a solve's
                                             end return at once and count too)                         */
} gofd_mmpde_kernel_stats;

typedef struct {
  double tau;        /* time scale of eq. x-1 (0: 1e-2)                                          */
  double t_end;      /* integrate over (0, t_end] (0: 1)                                           */
  double dt0;        /* first trial step (0: 1e-3)                                                 */
  int max_steps;     /* accepted steps at most (0: 400)                                            */
  double fixed_dt;   /* > 0: exactly max_steps steps of this length with no step control           */
  double gtol;       /* stop once |P grad I_h| <= gtol |P grad I_h(x_start)| (0: 1e-6)             */
  double cg_tol;     /* relative residual of each step's conjugate-gradient solve (0: 1e-10)      */
  int max_cg;        /* iterations of each solve at most (0: 20000)                               */
  gofd_mmpde_kernel_stats* stats;  /* host, nullable: kernel timings of the move                    */
} gofd_mmpde_opts;

typedef struct {
  int steps;              /* accepted steps                                                    */
  int rejected;           /* halvings of the step                                              */
  double t;               /* time reached                                                      */
  double energy_start;    /* I_h at the mesh given                                             */
  double energy_end;      /* I_h at the mesh returned                                          */
  int64_t cg_iterations;  /* conjugate-gradient iterations over all trial steps                */
  double grad_start;      /* |P grad I_h| at the mesh given (P: projection onto allowed motions) */
  double grad_end;        /* |P grad I_h| at the mesh returned                                 */
} gofd_mmpde_info;

/* Topology of the mesh: vertex two-rings, the elements around every vertex,
 * element neighbours and the boundary vertices, built on the host from
 * elems_dev (N_e x 3 int32, copied; every index in [0, N_v)).  *out is
 * library-owned, freed with gofd_mmpde_free.  Synchronises.
 * Errors: GOFD_E_ARG (N_v < 3, N_e < 1, an index out of range, a vertex in
 * no element, unknown boundary mode), GOFD_E_HIP, GOFD_E_OOM. */
int gofd_mmpde_create(gofd_ctx ctx, int64_t nv, int64_t ne, const int32_t* elems_dev, int boundary,
                      gofd_mmpde* out);
int gofd_mmpde_free(gofd_mmpde mm);

/* Vertex metrics of eq. MK-1 for u_dev on the mesh X_dev: the vertex Hessian
 * is that of the least-squares quadratic through u at the vertex's two-ring
 * (written to hess_dev when it is not NULL; a two-ring on which quadratics
 * are not unisolvent gives a zero Hessian), H_K the mean of its vertices'
 * Hessians, |H| = sqrt(H^2), alpha_h the root of sum_K |K| det(I + |H_K| /
 * alpha)^{1/3} = 2 |Omega| (bisection in log alpha to relative width 1e-15),
 * and M_i = det(I + |H_i| / alpha_h)^{-1/6} (I + |H_i| / alpha_h); when every
 * H_K vanishes alpha_h = +inf and M_i = I.  Writes Mv_dev (N_v x 3) and, when
 * alpha_host is not NULL, alpha_h.  Synchronises.
 * Errors: GOFD_E_ARG, GOFD_E_DEGENERATE (the elements' areas do not sum to a
 * positive value), GOFD_E_HIP, GOFD_E_OOM. */
int gofd_mmpde_metric(gofd_ctx ctx, gofd_mmpde mm, const double* X_dev, const double* u_dev, double* Mv_dev,
                      double* hess_dev, double* alpha_host);

/* I_h of eq. I-h for the mesh X_dev in the metric field of (Xb_dev, Mv_dev)
 * (walks start at each element's own index in the background mesh):
 * energy_host (nullable; +inf when an element has non-positive area), its
 * gradient dI_h/dx_i including the metric's variation (grad_dev, N_v x 2,
 * nullable; no boundary rule) and the element metrics M_K (MK_dev, N_e x 3,
 * nullable).  Synchronises. Errors: GOFD_E_ARG, GOFD_E_HIP, GOFD_E_OOM. */
int gofd_mmpde_energy(gofd_ctx ctx, gofd_mmpde mm, const double* Xb_dev, const double* Mv_dev, const double* X_dev,
                      double* grad_dev, double* MK_dev, double* energy_host);

/* Hessians of the elements' terms of I_h for the element metrics MK_dev held
 * fixed, with respect to their six vertex coordinates (x_0, y_0, x_1, y_1,
 * x_2, y_2), by central differences of the analytic element gradient with
 * the step 1e-5 times the element's longest edge, symmetrised: hess_dev is
 * N_e x 36 doubles (row-major 6 x 6 per element).  Asynchronous.
 * Errors: GOFD_E_ARG, GOFD_E_HIP. */
int gofd_mmpde_element_hessians(gofd_ctx ctx, gofd_mmpde mm, const double* X_dev, const double* MK_dev,
                                double* hess_dev);

/* Integrates eq. x-1, dx_i/dt = -sqrt(det M(x_i)) / tau dI_h/dx_i, with
 * Mv_dev the vertex metrics of the mesh X_dev given (its field on that mesh
 * for the whole move, sqrt(det M(x_i)) from Mv), in place on X_dev.  The
 * system is stiff; it is integrated by linearly implicit steps of length h:
 *     P (tau/h Q^{-1} + J) P dx = -P dI_h/dx,   Q = diag(sqrt(det M(x_i))),
 * P the projection onto the allowed motions, J the sum of the element
 * Hessians of gofd_mmpde_element_hessians for the current M_K, solved by
 * conjugate gradients with the vertices' 2 x 2 blocks as preconditioner.  A
 * trial step is halved until the solve converges with positive curvature
 * throughout, no element inverts and I_h decreases; the next trial step is
 * twice the accepted one, or the same after a halving.  Stops at t_end, after max_steps accepted steps,
 * once the projected gradient has fallen to gtol of its initial norm (the
 * flow is at rest), or when no step of at least 1e-6 times the longest
 * accepted one (and 1e-14) decreases I_h.  With opts->fixed_dt > 0 it takes
 * exactly max_steps steps of that length, with no energy test and no
 * gradient stop.  opts and info (host) are nullable.  The solver's
 * iterations go out in chunks of 8 whose state the host reads while the
 * next chunk runs; synchronises after every trial step.
 * Errors: GOFD_E_ARG, GOFD_E_DEGENERATE (the mesh given has an inverted
 * element), GOFD_E_BREAKDOWN (fixed_dt: a step system was not positive
 * definite), GOFD_E_HIP, GOFD_E_OOM. */
int gofd_mmpde_move(gofd_ctx ctx, gofd_mmpde mm, double* X_dev, const double* Mv_dev, const gofd_mmpde_opts* opts,
                    gofd_mmpde_info* info);

/* ---------------------------------------------------------------- GoFD in one dimension */

/* The 1D example of Section 5: the mesh of an interval is its vertices x_0 <
 * x_1 < .. < x_n (element e = [x_e, x_{e+1}], Dirichlet vertices x_0 and
 * x_n), the overlay grid has W = 2N+1 nodes z_k = (center - R) + k h, h = R/N
 * (each operation rounded separately), and T is the closed form of eq.
 * T-1D-0.  A node belongs to the element of smallest id whose closed
 * interval holds it (exact comparisons); nodes outside [x_0, x_n] have a zero
 * row.  A_FD is applied by its circulant embedding of length L = the smallest
 * power of two >= max(512, 4N) (eq. AU-1); L <= 4096 (N <= 1024), so that one
 * workgroup holds a line: products and whole CG solves run one workgroup per
 * field or right-hand side, one launch for all of them.  Vertex vectors have
 * N_v = n + 1 entries, grid vectors W; several fields or right-hand sides are
 * stored one after another.  FP64 throughout. */
typedef struct gofd1d_s* gofd1d;

typedef struct {
  int W;                  /* grid nodes                                                  */
  int L;                  /* FFT length                                                  */
  double h;               /* grid spacing R/N                                            */
  double a_h;             /* shortest element                                            */
  double dmin_interior;   /* min D_j over the interior vertices                          */
  int64_t n_inside;       /* nodes in an element                                         */
} gofd1d_info;

typedef struct {
  int iterations;         /* CG iterations                                               */
  double rel_residual;    /* ||r|| / ||b|| of the recursive residual at exit             */
  int converged;          /* 1 if ||r|| <= tol ||b||                                     */
} gofd1d_solve_info;

enum { GOFD1D_ELEM = 0, GOFD1D_WEIGHTS = 1, GOFD1D_D = 2, GOFD1D_T = 3 };

/* Transfer (location, weights, column sums D), T and the spectrum of its
 * embedding for the mesh x_dev (N_v doubles, strictly increasing; copied),
 * on the grid (N, R, center), order s in (0, 1).  *out is library-owned,
 * freed with gofd1d_free.  info (host, nullable).  Synchronises.
 * Errors: GOFD_E_ARG (N_v < 3, N < 1, R <= 0, s outside (0, 1), vertices
 * not increasing), GOFD_E_UNSUPPORTED (N > 1024), GOFD_E_RANK (2N+1 < N_v),
 * GOFD_E_ZERO_COLSUM (an interior vertex touches no node: grid too coarse),
 * GOFD_E_HIP, GOFD_E_OOM. */
int gofd1d_create(gofd_ctx ctx, int64_t nv, const double* x_dev, int N, double R, double center, double s,
                  gofd1d* out, gofd1d_info* info);
int gofd1d_free(gofd1d h);

/* Copy a part to out_dev: GOFD1D_ELEM (W int32, element of each node or -1),
 * GOFD1D_WEIGHTS (2W doubles: lambda_0, lambda_1 of each node, 0 outside),
 * GOFD1D_D (N_v doubles), GOFD1D_T (2N+1 doubles, T_0..T_2N).  Asynchronous.
 * Errors: GOFD_E_ARG, GOFD_E_HIP. */
int gofd1d_export(gofd_ctx ctx, gofd1d h, int part, void* out_dev);

/* y = D^{-1} I^T A_FD I u (eq. Ah-1; 0 where D = 0) for nfields fields of N_v
 * values (u at every vertex, used as given).  Asynchronous.
 * Errors: GOFD_E_ARG, GOFD_E_HIP, GOFD_E_OOM. */
int gofd1d_apply_Ah(gofd_ctx ctx, gofd1d h, int nfields, const double* u_dev, double* y_dev);

/* Solves eq. GoFD-2, (I^T A_FD I) u = h^{2s} I^T f on the interior vertices
 * (u = 0 at x_0 and x_n), for nrhs right-hand sides f given on the grid (W
 * values each), by CG from u = 0 (precond 0) or CG preconditioned by D_h
 * (precond 1), stopping when ||r|| <= tol ||b|| or after max_iter iterations
 * (<= 0: 10 N_v + 100).  Writes u_dev (nrhs x N_v) and info (host, nrhs
 * entries, nullable).  Synchronises.
 * Errors: GOFD_E_ARG, GOFD_E_NOT_CONVERGED (some right-hand side reached
 * max_iter; its best iterate is written), GOFD_E_BREAKDOWN, GOFD_E_HIP,
 * GOFD_E_OOM. */
int gofd1d_solve(gofd_ctx ctx, gofd1d h, int nrhs, const double* f_dev, double tol, int max_iter, int precond,
                 double* u_dev, gofd1d_solve_info* info);

#ifdef __cplusplus
}
#endif
#endif /* GOFD_H */
