/*
 * spi.h -- C ABI of the MI355X (gfx950) sparse weighted least-squares solver.
 *
 * The library solves the normal equations of a weighted linear
 * least-squares problem and returns the variances of the solution, as
 * stated in Bouchet et al., "Simultaneous analysis of large INTEGRAL/SPI
 * datasets" (Sect. 2.4.1, the chi-square merit function, the normal
 * equation and the variance relation):
 *
 *     A = H^T W H,   b = H^T W y,   x = A^-1 b,   Var(x_i) ~ (A^-1)_ii
 *
 * with H an M x N sparse transfer matrix, W = Sigma^-2 a positive diagonal
 * weight (one weight per measurement row) and y the data.  The solve is a
 * sparse direct method in three phases (Sect. 3.2): analysis on the host
 * (ordering and symbolic structure, Sect. 3.2.1), a multifrontal Cholesky
 * factorisation A = L L^T on the GPU (Sect. 3.2.2; D of the paper's L D L^T
 * is folded into L), and forward/backward substitution (Sect. 3.2.3).  The
 * variances are the diagonal of A^-1 (Sect. 3.3), computed by selected
 * inversion on the pattern of L.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Status: every call returns an int status (enum spi_status).  Nothing
 *    aborts or throws across the ABI.  spi_last_error() gives a text.
 *  - Ownership: the caller owns every buffer it passes.  The library copies
 *    what it keeps (the pattern during spi_analyze, the values during
 *    spi_set_values) into memory owned by the handle, freed by spi_destroy.
 *  - Memory: "host" pointers are ordinary CPU memory; "device" pointers are
 *    GPU memory of the device that was current at spi_analyze (for instance
 *    torch.Tensor.data_ptr() of a CUDA/HIP tensor).
 *  - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *    All device work of a handle is ordered on that stream.  Calls that
 *    only enqueue work (spi_set_values, spi_rhs, spi_solve, spi_diag_inv)
 *    return before it completes: device outputs are defined once the
 *    stream has reached that point, as with hipMemcpyAsync.  spi_factor
 *    synchronises the stream before returning, because it reports a
 *    non-positive pivot as a status.
 *  - Threads: one handle must not be used by two threads at once.
 *  - Indices are 0-based.  Dense vectors are float64, in the original
 *    unknown order (column order of H) unless stated otherwise.
 */
#ifndef SPI_H
#define SPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spi_handle spi_handle;

enum spi_status {
    SPI_OK = 0,
    SPI_E_ARG = 1,      /* invalid argument / malformed CSR / unobserved unknown */
    SPI_E_STATE = 2,    /* call out of order (e.g. spi_solve before spi_factor) */
    SPI_E_NOT_SPD = 3,  /* a non-positive or non-finite pivot (A not SPD) */
    SPI_E_OOM = 4,      /* device allocation failed */
    SPI_E_HIP = 5,      /* any other HIP runtime error */
    SPI_E_NOCONV = 6    /* iterative refinement did not reach its tolerance */
};

enum spi_precision {
    SPI_FP64 = 0,       /* every stage in binary64 */
    SPI_MIXED = 1       /* the rank-k updates of the root front (the bulk
                           and lookahead updates of the block sweeps, or
                           with root_inverse = 0 the Cholesky and factor
                           inversion products) on the binary32 matrix
                           cores: every binary32 sum runs over at most 256
                           terms and such sums add up in binary64;
                           binary64 storage, pivot blocks, band products,
                           leaf fronts, refinement residuals and the leaf
                           selected-inversion sums */
};

typedef struct spi_opts {
    int32_t precision;      /* enum spi_precision; default SPI_FP64 */
    int32_t max_group;      /* max leaf columns amalgamated in one front (and
                               rows in one row panel); default 32.  A panel of
                               (k + 24) (|U| + 32) 8 bytes or more is rejected
                               by the analysis (32-bit offsets) */
    double leaf_max_work;   /* a column is a leaf candidate only if the total
                               length of the rows it appears in is <= this;
                               default 65536 */
    double amalg_density;   /* min fraction of structural non-zeros in an
                               amalgamated leaf panel; default 0.35 */
    int32_t refine_steps;   /* refinement steps of spi_solve with a
                               double-double residual; default 1 (on the
                               medium workload x is within 1.1e-13 of the
                               certified solution with none, 8.5e-14 with
                               one, and a second changes nothing) */
    int32_t timing;         /* 1: time the phases with HIP events on the
                               handle's stream (see spi_info); default 0 */
    int32_t root_inverse;   /* 1: spi_factor inverts the dense root front
                               by block sweeps (Gauss-Jordan on the
                               symmetric Schur complement, the Cholesky
                               pivot blocks), so the root block of A^-1 is
                               ready for spi_diag_inv and spi_solve applies
                               it as a symmetric product; 0: spi_factor
                               computes the Cholesky factor, spi_solve
                               substitutes, and spi_diag_inv inverts the
                               factor and forms W^T W.  Default 1 */
    int32_t equilibrate;    /* 1: factor S A S with S = diag(s), s_c the power
                               of two 2^-floor(log2(A_cc)/2) (scaled diagonal
                               in [1, 4)); exact, so FP64 results do not
                               change, and it keeps the FP32 stages of
                               SPI_MIXED in range; 0: no scaling.  Default 1 */
    double refine_tol;      /* > 0: spi_solve stops refining once the
                               max-norm of the correction is <= refine_tol
                               times the max-norm of x, or once the last two
                               corrections contract (by at least half) at a
                               rate that puts the next one below that
                               (reading the norms back synchronises the
                               stream after each step), and returns
                               SPI_E_NOCONV if refine_steps steps do not get
                               there; 0: exactly refine_steps steps.
                               Default 0; SPI_MIXED uses 1e-14 and at least
                               10 steps when this is 0 */
    int32_t keep_root_order;/* 0: the analysis numbers the root unknowns
                               for locality (columns that share many rows
                               end up in the same 64-column tiles, so fewer
                               tiles of the dense root see each row); 1:
                               original order.  Default 0 */
    int32_t leaf_lds_cap;   /* widest leaf front (root positions) whose
                               panel columns are accumulated in on-chip
                               memory (LDS) before one write; wider fronts
                               accumulate in place in device memory.  0:
                               2048 (the most LDS allows); 1..2048 a
                               smaller cap (tests use it to run the in-place
                               path on small problems) */
    int32_t selinv_chunk;   /* tasks (64 x 64 blocks of a front's row
                               structure) per launch of the leaf selected
                               inversion.  0: 4194304 (a launch must stay
                               below 2^24 workgroups); >= 1 a smaller chunk
                               (tests use it to run several launches) */
    int32_t keep_root_sum;  /* 1: the handle keeps A_RR, the root block of
                               H^T W H (one more n_pad^2 buffer), so that a
                               factorisation after spi_set_leaf_values
                               re-assembles only the leaf fronts' updates
                               (Sect. 4.1, modified columns of H; App. A.5,
                               the empty-field loop).  Default 0 */
    int32_t indefinite;     /* 1: A may be symmetric indefinite (weights of
                               either sign; Sect. 5: the SPI matrices are,
                               numerically, and need 2 x 2 pivots; Sect.
                               3.2.2 and 4.3: the factorisation must pivot).
                               The root front's pivot blocks (64 columns)
                               are swept with Bunch-Kaufman 1 x 1 and 2 x 2
                               pivots of either sign chosen inside the
                               block; a block with no usable pivot is
                               reported as SPI_E_NOT_SPD at its first
                               column.  Row panels carry the weights'
                               signs.  Leaf pivots (A_cc of a leaf column)
                               must still be positive: a column whose pivot
                               is not is reported as before (it would have
                               to move into the root).  Needs
                               root_inverse = 1.  Default 0: positive
                               definite, every pivot checked */
    int32_t asm_tile;       /* edge of the root tiles summed on chip by the
                               root assembly: 64 or 128; 0 (default): 128
                               for roots of padded order 8192 and more, 64
                               below (four times the workgroups for small
                               fronts) */
    int64_t device_mem_cap; /* > 0: most device memory (bytes) spi_analyze /
                               spi_analyze_like may allocate for the handle
                               (the analysis maps and every work buffer they
                               size; spi_info.device_bytes reports what a
                               handle holds): a handle that needs more is
                               refused with SPI_E_OOM before any allocation
                               beyond the cap, and nothing is left
                               allocated.  0 (default): no cap */
    int32_t fp64_fallback;  /* 1: with SPI_MIXED, a spi_factor that meets a
                               non-positive pivot, or a spi_solve whose
                               refinement does not reach refine_tol (the
                               binary32 products too coarse for the
                               system's conditioning), is redone with every
                               stage in binary64: the root refactored, the
                               solve repeated (b must not overlap x); the
                               handle stays in binary64 until the next
                               spi_set_values or spi_set_leaf_values, and
                               spi_info.fp64_fallbacks counts the switches.
                               In spi_batch_run such a system is redone
                               alone in binary64 after the batch's
                               synchronisation (outside any graph; its
                               graph is captured again at the next run).
                               0 (default): the call returns
                               SPI_E_NOT_SPD / SPI_E_NOCONV */
} spi_opts;

typedef struct spi_info_t {
    int64_t m, n, nnz_h;        /* shape of H and its non-zeros */
    int64_t nnz_a;              /* non-zeros of A = H^T W H (both triangles);
                                   -1 when counting them would cost more
                                   than 2e10 visits (sum of squared row
                                   lengths of H) */
    int64_t nnz_l;              /* non-zeros of L (lower, incl. diagonal, as stored) */
    int64_t n_leaf;             /* unknowns eliminated in leaf fronts */
    int64_t n_groups;           /* leaf fronts (amalgamated supernodes) */
    int64_t n_root;             /* order of the dense root front */
    int64_t n_root_padded;      /* root order padded to the tile size */
    int64_t failed_col;         /* original column of the first bad pivot, or -1 */
    double flops_factor;        /* algorithmic flops of spi_factor */
    double flops_selinv;        /* algorithmic flops of spi_diag_inv */
    double flops_solve;         /* algorithmic flops of one spi_solve pass, 1 RHS */
    double flops_assembly;      /* flops of the H^T W H assembly */
    double t_analyze_ms;        /* host time of spi_analyze */
    int32_t precision;          /* precision in use */
    int32_t refine_steps_done;  /* refinement steps of the last spi_solve */
    double last_refine_norm;    /* max-norm of the last correction / max-norm of x */
    /* Device time of the phases of the last calls, in ms, measured with HIP
     * events on the handle's stream when opts.timing = 1 (else 0): */
    double t_leaf_ms;           /* leaf fronts: assembly, pivots, panels */
    double t_extend_ms;         /* root assembly + extend-add of the leaves */
    double t_potrf_ms;          /* root Cholesky, or the root inversion by
                                   block sweeps (root_inverse = 1) */
    double t_solve_ms;          /* whole spi_solve incl. refinement */
    double t_trtri_ms;          /* inverse of the root factor */
    double t_lauum_ms;          /* root block of A^-1 from the inverse factor */
    double t_selinv_ms;         /* leaf selected inversion + diagonal output */
    /* The bulk updates of the root inversion by block sweeps
     * (root_inverse = 1; one symmetric rank-kb product per column band): */
    double t_sweep_bulk_ms;     /* device time of the bulk updates */
    double flops_sweep_bulk;    /* their algorithmic flops (lower triangles
                                   only), summed over the timed calls */
    /* Flops the kernels execute, zeros of the dense panels included (the
     * algorithmic counts above take the exact column counts of L): */
    double flops_exec_assembly; /* root assembly: sum over the panels'
                                   incidences on the 64 x 64 root tiles of
                                   2 nI nJ k */
    double flops_exec_selinv;   /* leaf selected inversion: sum over its
                                   tasks of 2 na nb p */
    double flops_root_assembly; /* algorithmic flops of the root front's
                                   assembly: the lower triangles of the row
                                   products w_r h_rR h_rR^T and of the leaf
                                   updates L_Ul L_Ul^T on the exact
                                   structure, len (len + 1) per row or leaf */
    int32_t root_assembly_mode; /* last spi_factor's root assembly: 0 all
                                   panels, 1 all panels keeping A_RR
                                   (opts.keep_root_sum), 2 the kept A_RR
                                   plus the leaf fronts (after
                                   spi_set_leaf_values) */
    int32_t asm_tile;           /* root assembly tile edge (64 or 128) */
    int64_t device_bytes;       /* device memory the handle holds: analysis
                                   maps and work buffers sized by
                                   spi_analyze (not the learned
                                   preconditioner's, nor the library's fixed
                                   scratch array); 0 from spi_symbolic */
    int32_t fp64_fallbacks;     /* opts.fp64_fallback: switches from
                                   SPI_MIXED to binary64 so far */
} spi_info_t;

/* Fill `o` with the defaults listed above. */
void spi_default_opts(spi_opts* o);

/*
 * Analysis (Sect. 3.2.1): validate the pattern of H, choose the
 * elimination order, build the assembly tree (independent leaf fronts whose
 * unknowns share no measurement row, amalgamated into supernodes, and one
 * dense root front), the index maps the kernels use, and upload them.
 *
 *  h       [out] new handle (NULL on failure, except SPI_E_ARG detail text
 *                is not available then; spi_last_error(NULL) returns the
 *                last analysis error of the calling thread)
 *  m, n    rows (measurements) and columns (unknowns) of H; m >= 1, n >= 1
 *  rowptr  host, int64[m + 1], CSR row pointers, rowptr[0] = 0, non-decreasing
 *  col     host, int32[rowptr[m]], column indices, strictly increasing
 *          within each row, each in [0, n)
 *  opts    host, may be NULL for the defaults
 *  stream  hipStream_t for all device work of this handle
 *
 * Errors: SPI_E_ARG for a malformed pattern or an unknown that appears in no
 * row (A would be singular); SPI_E_OOM / SPI_E_HIP on device failures.
 */
int spi_analyze(spi_handle** h, int64_t m, int64_t n, const int64_t* rowptr,
                const int32_t* col, const spi_opts* opts, void* stream);

/*
 * Numerical values on the analysed pattern (one energy band): H's values in
 * CSR order and the row weights W = Sigma^-2 (Sect. 2.4.1).  Stream-ordered
 * device-to-device copy into handle-owned buffers; invalidates any factor.
 *
 *  val  device, float64[nnz(H)], finite
 *  w    device, float64[m], finite.  The paper's weights are positive
 *       (inverse variances).  Zero and negative weights are accepted: a zero
 *       weight drops a row (the Hessian of the likelihood fit has weight
 *       d_r / e_r^2, zero where no count was recorded), a negative one
 *       removes a row's contribution; A may then be singular or indefinite,
 *       which spi_factor reports as SPI_E_NOT_SPD.
 * The values are checked on the device, without a synchronisation here: a
 * NaN or infinite value or weight makes the next spi_factor (or batch run)
 * return SPI_E_ARG.
 */
int spi_set_values(spi_handle* h, const double* val, const double* w);

/*
 * New values of H in the leaf-front columns only (in the coded-mask model,
 * the background columns, the first K0 columns of H: App. A.5 updates them
 * at each pass of the empty-field loop; Sect. 4.1 times such updates of
 * A = H^T H).  `val` is a full device array like spi_set_values' (float64
 * [nnz(H)], finite); the weights are kept.  The root block of A does not
 * depend on leaf columns, so with opts.keep_root_sum = 1 the next
 * spi_factor starts from the kept A_RR and assembles only the leaf fronts'
 * updates.  The call compares the root entries of `val` with the values in
 * use; if any differs, the next spi_factor assembles everything again (the
 * result is right either way).  SPI_E_STATE before spi_set_values.
 * Stream-ordered; invalidates any factor.
 */
int spi_set_leaf_values(spi_handle* h, const double* val);

/*
 * Numerical factorisation (Sect. 3.2.2): assembles A = H^T W H directly into
 * the leaf fronts and the root front (extend-add of the leaf contribution
 * blocks), factors the leaf fronts, then treats the dense root: with
 * opts.root_inverse = 1 (default) it is inverted in place by block sweeps,
 * whose pivot blocks are those of its Cholesky factorisation; with 0 it is
 * Cholesky-factored.  Synchronises the handle's stream.  Returns
 * SPI_E_NOT_SPD if a pivot is not positive (the same pivot on either
 * route); spi_info().failed_col then names the original column.
 * SPI_E_STATE before spi_set_values; SPI_E_ARG if the values or weights of
 * the last spi_set_values hold a NaN or an infinity (no factor is left).
 */
int spi_factor(spi_handle* h);

/*
 * Right-hand side of the normal equations b = H^T W y (Sect. 2.4.1).
 *  y  device, float64[m]       b  device, float64[n] (written)
 */
int spi_rhs(spi_handle* h, const double* y, double* b);

/*
 * Solve A x = b by forward and backward substitution over the assembly tree
 * (Sect. 3.2.3; at the root, one product with the root block of A^-1, or
 * substitution with its Cholesky factor when root_inverse = 0), followed by
 * opts.refine_steps steps of iterative refinement whose residual
 * b - H^T W (H x) is accumulated in double-double arithmetic from H itself.
 *  b     device, float64, column-major n x nrhs with leading dimension ldb
 *  x     device, float64, same layout (written); may not alias b
 *  nrhs  >= 1;  ldb >= n
 * SPI_E_STATE if no valid factor.
 */
int spi_solve(spi_handle* h, const double* b, double* x, int32_t nrhs,
              int64_t ldb);

/*
 * Variances: d_i = (A^-1)_ii for every unknown, original order, unscaled
 * (Sect. 2.4.1 variance relation; Sect. 3.3 partial computation of the
 * inverse).  Computed by selected inversion on the pattern of L: the full
 * inverse of the root front (already formed by spi_factor's sweeps, or by
 * inverting its Cholesky factor when root_inverse = 0), then for every leaf
 * front the entries it needs.
 *  d  device, float64[n] (written)
 * SPI_E_STATE if no valid factor.
 */
int spi_diag_inv(spi_handle* h, double* d);

/*
 * General entries of A^-1, e.g. covariances between unknowns (Sect. 3.3.1:
 * the entries a^-1_ij of the inverse that are requested; the diagonal gives
 * the variances).  out[q] = (A^-1)_{rows[q], cols[q]}, original unknown
 * order, unscaled.  Every entry is computed from the root block of A^-1
 * (formed by spi_factor's sweeps, or from the Cholesky factor on the first
 * call when root_inverse = 0) and the leaf panels, by the same relations as
 * the selected inversion, one workgroup per entry: an entry between two
 * leaf unknowns costs |U_g| |U_h| products (the root positions of their
 * fronts), one with a root unknown |U_g|.
 *  k           number of entries (>= 0)
 *  rows, cols  device int32[k], each in [0, n) (copied to the host and
 *              checked: SPI_E_ARG otherwise; this synchronises the stream)
 *  out         device float64[k] (written)
 * SPI_E_STATE without a valid factor.
 */
int spi_inv_entries(spi_handle* h, int64_t k, const int32_t* rows,
                    const int32_t* cols, double* out);

/*
 * spi_diag_inv for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result as spi_diag_inv, with the selected
 * inversion's partial sums in a fixed array of device memory inside the
 * library instead of the handle's buffer.  The call allocates and creates
 * nothing (no phase timing even with opts.timing; it needs a factor from a
 * successful spi_factor, which has created everything else it uses).
 *  d  device, float64[n] (written)
 * The array holds 2^23 doubles (64 MiB) on each GPU the library runs on,
 * kept until the process ends; a handle whose selected inversion needs more
 * (about 38 MiB for the medium workload, far more for the large one) gets
 * SPI_E_ARG.  All calls on one GPU share that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must not be
 * issued.  SPI_E_STATE without a valid factor.
 */
int spi_diag_inv_noalloc(spi_handle* h, double* d);

/*
 * The analysis phase alone, on the host, with no device work (Sect. 3.2.1):
 * useful to size a problem before allocating it, and to inspect the
 * elimination order and tree.  Same pattern arguments and errors as
 * spi_analyze.  `info` (may be NULL) receives the analysis counters (the
 * fields of the last calls stay zero).  If non-NULL:
 *   elim_order  host int32[n]: original columns in elimination order
 *               (leaf fronts first, then the root front)
 *   col_parent  host int32[n]: parent of each original column in the column
 *               elimination tree of the stored factor (the first later
 *               column with a non-zero in its column of L), -1 for the root
 *   front_of    host int32[n]: leaf front of each column, -1 for root columns
 */
int spi_symbolic(int64_t m, int64_t n, const int64_t* rowptr,
                 const int32_t* col, const spi_opts* opts, spi_info_t* info,
                 int32_t* elim_order, int32_t* col_parent, int32_t* front_of);

/*
 * Checkpoint of the analysis (Sect. 3.2.1: the ordering and symbolic
 * factorisation are done once per pattern; later runs on the same pattern
 * skip them).  The files are binary, of this library's own format (a
 * version tag, every array of the analysis with its length, a 64-bit hash);
 * reading refuses a missing, truncated, corrupted or foreign file with
 * SPI_E_ARG (spi_last_error(NULL) says why, or spi_last_error(h) for
 * spi_save_analysis) before anything reaches the device.
 *
 * spi_save_analysis     write the analysis of handle h (and the analysis
 *                       options that shaped it: max_group, leaf_max_work,
 *                       amalg_density, keep_root_order, asm_tile) to path.
 * spi_symbolic_save     host only: analyse the pattern as spi_symbolic
 *                       does and write the file (no device needed).
 * spi_analysis_file_info host only: read and check a file; fill `info` with
 *                       its counters as spi_symbolic does.
 * spi_analyze_load      a new handle from a file, as spi_analyze from the
 *                       same pattern: opts may be NULL (defaults); their
 *                       analysis options are replaced by the file's.  The
 *                       handle holds the file's pattern (H's rowptr and col)
 *                       and is then used exactly as one from spi_analyze.
 */
int spi_save_analysis(const spi_handle* h, const char* path);
int spi_symbolic_save(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                      const spi_opts* opts, const char* path);
int spi_analysis_file_info(const char* path, spi_info_t* info);
int spi_analyze_load(spi_handle** h, const char* path, const spi_opts* opts,
                     void* stream);

/*
 * A new handle on the same pattern as `src` (another energy band, Sect.
 * 2.2.3): the host analysis of `src` is copied instead of recomputed, then
 * uploaded and the device buffers sized as in spi_analyze.
 *  opts    may be NULL (src's options as created: the precision asked
 *          for, not a binary64 fallback src has made); the analysis options (max_group,
 *          leaf_max_work, amalg_density, keep_root_order, asm_tile) must
 *          equal src's
 *  stream  hipStream_t of the new handle
 */
int spi_analyze_like(spi_handle** h, const spi_handle* src, const spi_opts* opts,
                     void* stream);

/* Counters of the analysis and of the last calls; with opts.timing the
 * accumulated phase times since spi_analyze (synchronises the stream).
 * Host struct. */
int spi_info(const spi_handle* h, spi_info_t* info);

/* Text of the last error of `h` (or of the calling thread's last
 * spi_analyze if h is NULL).  Valid until the next call on h. */
const char* spi_last_error(const spi_handle* h);

/* Free the handle and all its device memory (synchronises its stream). */
void spi_destroy(spi_handle* h);

/* ------------------------------------------------------------------------
 * Learned preconditioner for many bands on one pattern
 * ------------------------------------------------------------------------
 * The energy bands of one observation share the pattern of H and differ in
 * W and y (Sect. 2.2.3).  Iterative methods need a good preconditioner to
 * converge (Sect. 3.1).  Here the direct factor of a reference band r
 * (a handle after spi_factor) preconditions conjugate gradients on a later
 * band b.  A small network corrects it with a per-unknown diagonal:
 *
 *     M^-1 = D A_r^-1 D,   D = diag(d),   d_j = exp(g(f_j))
 *
 * Features of unknown j:
 *     f0 = log(A_b,jj / A_r,jj)
 *     f1 = 1 for a root-front unknown, else 0
 *     f2 = mean of f0 over the unknowns of the same kind
 * Network (hidden width HID in {8, 16, 32}, binary32, shared by all unknowns):
 *     h1 = tanh(W1 f + b1),  h2 = tanh(W2 h1 + b2),  g = w3.h2 + b3 + wl.f
 * Parameters are stored flat, in binary32, in this order:
 *     W1 (HID x 3, row-major), b1 (HID), W2 (HID x HID, row-major),
 *     b2 (HID), w3 (HID), b3 (1), wl (3)
 * Training loss on a band with direct solution x of A_b x = rhs:
 *     L = e^T A_b e / (2 x^T rhs),   e = M^-1 rhs - x
 * The forward and backward passes and the Adam update run on the GPU.
 * Every call below runs on the band handle's stream.  The reference handle
 * must use the same stream and the same pattern.
 */
typedef struct spi_lp spi_lp;

/* Number of parameters for hidden width `hidden`, or -1 if unsupported. */
int64_t spi_lp_param_count(int32_t hidden);

/* New network with the given initial parameters (host, binary32,
 * spi_lp_param_count(hidden) values, layout above); Adam state zero. */
int spi_lp_create(spi_lp** lp, int32_t hidden, const float* params);

/* Copy the current parameters to `params` (host, binary32). */
int spi_lp_get_params(const spi_lp* lp, float* params);

/*
 * Training loss of one band, and optionally its gradient.
 *  band  handle with the band's values (spi_set_values)
 *  ref   factored reference handle
 *  rhs   device, float64[n]: right-hand side of the band
 *  x     device, float64[n]: its direct solution
 *  loss  host, written
 *  grad  host, float64[param_count] or NULL: dL/dparams (synchronises)
 * Costs two solves with the reference factor and one product with A_b.
 */
int spi_lp_loss_grad(spi_lp* lp, spi_handle* band, spi_handle* ref,
                     const double* rhs, const double* x, double* loss,
                     double* grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on one band's loss, with
 * learning rate lr; `loss` (host) receives the loss before the step. */
int spi_lp_train_step(spi_lp* lp, spi_handle* band, spi_handle* ref,
                      const double* rhs, const double* x, double lr,
                      double* loss);

void spi_lp_destroy(spi_lp* lp);

typedef struct spi_pcg_info {
    int32_t iterations;     /* inner binary32 CG iterations, all passes */
    int32_t outer;          /* binary64 residual passes */
    int32_t fell_back;      /* 1: tolerance not met, solved by spi_factor +
                               spi_solve on the band instead */
    int32_t reserved;
    double rel_residual;    /* ||b - A x||_2 / ||b||_2 of the returned x, binary64 */
} spi_pcg_info;

/*
 * Solve A_b x = b by preconditioned conjugate gradients with M^-1 above
 * (lp = NULL: no correction, d = 1).  The method is iterative refinement in
 * binary64: each pass takes the true residual r = b - A_b x, accumulated in
 * double-double from H.  Within a pass, conjugate gradients in binary32
 * solve A_b e = r to a relative residual of 1e-5, with products by H and
 * H^T in binary32; the preconditioner applies the reference factor's
 * binary64 solves.  Then x += e.
 * Stops when ||b - A_b x|| <= tol ||b|| (binary64).
 * If `maxit` inner iterations do not get there, the band is factored and
 * solved directly (its own multifrontal factor) and `fell_back` is set;
 * if even that x misses `tol`, the call returns SPI_E_NOCONV (x and `info`
 * are still written).
 *  b, x  device, float64[n];  tol > 0;  maxit >= 1
 *  info  host, may be NULL
 * Synchronises the stream (the scalars of CG are read back every iteration).
 */
int spi_pcg_solve(spi_handle* band, spi_handle* ref, const spi_lp* lp,
                  const double* b, double* x, double tol, int32_t maxit,
                  spi_pcg_info* info);

/* ------------------------------------------------------------------------
 * Empty-field loop: the detector pattern computed with the solution
 * ------------------------------------------------------------------------
 * App. A.4-A.5.  In the paper's background model (Sect. 2.2.3) the
 * background column of row i = (pointing p, detector d) holds U_u t_i: t_i
 * the effective time, U_u the detector pattern of the row's unit u (its
 * detector, or (detector, interval of pointings) for the per-interval
 * variant), and x at that column the background intensity of the time bin.
 * With x fixed, the pattern that minimises chi^2 for each unit is
 *     LSQ: U_u = sum (y_i - D^S_i) g_i w_i / sum g_i^2 w_i,
 *     MLE: U_u = sum (y_i - D^S_i) / sum g_i,
 * sums over the unit's rows, g_i = x_bg(i) t_i, D^S_i the source part of
 * (H x)_i and w_i the handle's weights (sigma_i^-2).  Arguments shared by
 * both calls (all device memory unless stated):
 *  val       float64[nnz(H)], H's values as given to spi_set_values (not
 *            equilibrated); its background entries are rewritten
 *  y         float64[m], the data
 *  bg_pos    int64[m], CSR position of row i's background entry, -1 if none
 *  t         float64[m], t_i
 *  grp_ptr   int64[n_u + 1], grp_rows int32[grp_ptr[n_u]]: the rows of each
 *            unit (CSR)
 *  stat      0: LSQ, 1: MLE update
 *  U         float64[n_u], the pattern (a unit whose rows give a zero
 *            denominator keeps its value)
 * Every sum runs in a fixed order, so results repeat bit for bit.
 */

/* One pattern update: chi2 (host, may be NULL) receives
 * sum_i w_i (y_i - (H x)_i)^2 with `val` as given; then U is updated and the
 * background entries of val set to U_u t_i.  Synchronises (chi2 read back).
 *  x  float64[n], the current solution */
int spi_empty_field_update(spi_handle* h, double* val, const double* y,
                           const double* x, const int64_t* bg_pos, const double* t,
                           const int64_t* grp_ptr, const int32_t* grp_rows,
                           int32_t n_u, int32_t stat, double* U, double* chi2);

/* Algorithm 1 (App. A.5).  The handle has had spi_set_values (the weights
 * and the sky columns' values are taken from there).  Each pass sets the
 * background entries to U_u t_i (spi_set_leaf_values: with
 * opts.keep_root_sum = 1 the root front is re-assembled from the kept
 * A_RR), factors, solves the LSQ problem for x (b = H^T W y), and takes
 * chi^2 of that x; passes stop once chi^2 decreases by no more than rtol
 * times its previous value, or after itermax passes; between passes U gets
 * the closed-form update from x.  On return x, U and val are those of the
 * last pass, d its variances diag(A^-1) (d may be NULL).
 *  itermax >= 1, rtol >= 0
 *  x          float64[n] (written)       d  float64[n] (written) or NULL
 *  chi2_hist  host float64[itermax] or NULL: chi^2 of every pass
 *  passes     host, may be NULL: passes run
 */
int spi_empty_field_loop(spi_handle* h, double* val, const double* y,
                         const int64_t* bg_pos, const double* t,
                         const int64_t* grp_ptr, const int32_t* grp_rows, int32_t n_u,
                         int32_t stat, int32_t itermax, double rtol, double* U,
                         double* x, double* d, double* chi2_hist, int32_t* passes);

/* ------------------------------------------------------------------------
 * Poisson likelihood fit (low counts): Newton's method on the solver
 * ------------------------------------------------------------------------
 * App. A.1-A.2.  With the model e = H x and counts y, the fit minimises
 * C = 2 sum_i (e_i - y_i ln e_i) (the likelihood of App. A.1 with its sign
 * turned; a row with y_i = 0 adds 2 e_i).  Its gradient is
 * G = 2 H^T (1 - y/e) and half its Hessian H^T [y/e^2] H, the normal matrix
 * of the same pattern with weights y_i / e_i^2, so every Newton step is a
 * factorisation and a solve of this library.
 *  val  device float64[nnz(H)], H's values (as given to spi_set_values)
 *  y    device float64[m], the counts (>= 0)
 */

/* Terms at x (device float64[n]): cash (host, may be NULL) = C; w (device
 * float64[m]) = y / e^2; g (device float64[n]) = H^T (y/e - 1) = -G/2, the
 * Newton right-hand side (computed with the handle's values, which must be
 * `val`).  SPI_E_ARG (cash = +inf) if some e_i <= 0.  Synchronises. */
int spi_mle_terms(spi_handle* h, const double* val, const double* y, const double* x,
                  double* w, double* g, double* cash);

/* Newton's method from x (device float64[n], in: the start, e.g. the LSQ
 * solution, App. A.2; out: the fit).  Each step sets the weights y/e^2
 * (spi_set_values), factors, solves for the step dx from H^T (y/e - 1), and
 * takes x + a dx: a = 1, halved while some e_i <= 0 or while C does not fall
 * by at least 1e-4 a |G . dx| (taken whole once the predicted decrease
 * |G . dx| is below 1e-12 |C|, which C cannot resolve).  Stops after a
 * step with max|a dx| <= tol max|x|, or after itermax steps.  d (device
 * float64[n] or NULL): diag of the inverse Hessian at the fit (App. A.2),
 * after which the handle holds the Hessian's weights.
 *  cash_hist  host float64[itermax + 1] or NULL: C at the start and after
 *             every step;   steps  host, may be NULL: steps taken
 * SPI_E_ARG if the start's model is not positive; SPI_E_NOCONV if the line
 * search halves the step below 1e-10.  Synchronises. */
int spi_mle_newton(spi_handle* h, const double* val, const double* y, double* x,
                   int32_t itermax, double tol, double* d, double* cash_hist,
                   int32_t* steps);

/* ------------------------------------------------------------------------
 * Batches: many systems in flight together
 * ------------------------------------------------------------------------
 * The paper analyses its energy bands one after the other, as many
 * sequential computations (Sect. 5: 24 consecutive bands; Sect. 6).  A
 * batch takes k handles of any patterns, each on its own stream (bands
 * from spi_analyze_like, independent sub-problems from spi_analyze).  It
 * enqueues each system's whole pipeline and synchronises once per stream
 * at the end, so the systems overlap on the GPU.
 */
typedef struct spi_batch spi_batch;

/* Group k distinct handles.  use_graphs = 1: on its first run, each
 * handle's pipeline is captured into a HIP graph.  Later runs with the
 * same buffer pointers and precision replay the graph; new pointers (or a
 * switch to binary64, see opts.fp64_fallback) re-capture it.  The launch
 * shapes are those of the capture: set the outer block and bulk tile
 * (spi_autotune, spi_set_potrf_block, spi_set_bulk_tile) before the first
 * run.  This needs non-NULL streams.  The handles stay owned by the caller
 * and must outlive the batch. */
int spi_batch_create(spi_batch** b, spi_handle* const* hs, int32_t k,
                     int32_t use_graphs);

/*
 * For each system i (values already set with spi_set_values):
 *  - spi_factor;
 *  - rhs[i] = H^T W y[i];
 *  - x[i] = A^-1 rhs[i], with exactly opts.refine_steps refinement steps
 *    (no read-back between steps inside a batch);
 *  - d[i] = diag(A^-1).
 * y, rhs, x, d: host arrays of k device pointers.  d may be NULL, as may
 * any d[i], to skip the variances.  status: host int32[k] or NULL, each
 * system's status (SPI_E_NOT_SPD etc.).  With opts.refine_tol > 0 (always
 * so in SPI_MIXED) the sizes of the last two corrections are read back at
 * the final synchronisation, and a system whose refinement did not reach
 * refine_tol by the rule of spi_solve gets SPI_E_NOCONV (x is still
 * written); with opts.fp64_fallback such a system, or one that met a
 * non-positive pivot in SPI_MIXED, is first redone alone in binary64 (see
 * spi_opts).  Returns SPI_OK, or the first failing status.  All systems
 * are finished on return.
 */
int spi_batch_run(spi_batch* b, const double* const* y, double* const* rhs,
                  double* const* x, double* const* d, int32_t* status);

void spi_batch_destroy(spi_batch* b);

/*
 * Autotuner of the root front's launch shapes: the outer block (the band
 * width of the block sweeps, or of the Cholesky's trailing updates: 128,
 * 256 or 512 columns, and 1024 for the sweeps in SPI_FP64 on roots of
 * padded order 1024 or more; one band or panel of lookahead) and, for the sweeps
 * on roots up to order 8192, the tile of their bulk update (128 x 128 or
 * 64 x 64: a small root gets four times the workgroups from the smaller
 * tile).  It times spi_factor on the handle's current values with each
 * candidate pair, keeps the fastest, and leaves a factor computed with it.
 *  chosen  host, may be NULL: the outer block chosen
 */
int spi_autotune(spi_handle* h, int32_t* chosen);
/*
 * Test aid: overwrite every device work buffer of the handle (values,
 * fronts, root, bands, partial sums, flags; not the analysis maps) with
 * 0xff bytes (NaN as binary64), so that a test can show that no result
 * depends on what a buffer held before.  Stream-ordered on the handle's
 * stream.  The handle then needs spi_set_values and spi_factor again.
 * Returns SPI_E_ARG for a NULL handle, SPI_E_HIP on a runtime error.
 */
int spi_debug_poison(spi_handle* h);

/* Current outer block of the root front, or -1 for a NULL handle. */
int spi_get_potrf_block(const spi_handle* h);
/* Tile edge of the sweeps' bulk update (64 or 128; default 128), or -1. */
int spi_get_bulk_tile(const spi_handle* h);
/* Set it by hand: 64 or 128. */
int spi_set_bulk_tile(spi_handle* h, int32_t tile);
/* Set the outer block by hand: 128, 256 or 512, or 1024 for the sweeps
 * (root_inverse = 1) in SPI_FP64 on a root of padded order 1024 or more
 * (fewer, wider bands: the bulk updates read and write the root half as
 * often); SPI_E_ARG otherwise.  SPI_MIXED with root_inverse = 0 uses at
 * most 256, the longest binary32 accumulation it allows; the sweeps split
 * longer products into launches of 256. */
int spi_set_potrf_block(spi_handle* h, int32_t block);

#ifdef __cplusplus
}
#endif

#endif /* SPI_H */
