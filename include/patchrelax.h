/*
 * patchrelax.h -- C ABI of the MI355X (gfx950) compressed patch-relaxation
 * library (libpatchrelax.so).
 *
 * Method: Harper & Tuminaro, "Compression and Reduced Representation
 * Techniques for Patch-Based Relaxation" (arXiv 2306.10025).
 *   - patches, restriction V_k, patch matrices A_k = V_k A V_k^T and the
 *     averaging weight W: Section 2;
 *   - patch preconditioner M^{-1} = W sum_k V_k^T A_k^{-1} V_k: Eq.(1);
 *   - approximate (compressed) preconditioner with an inverse database and a
 *     map phi, M~^{-1} = W sum_k V_k^T B_phi(k)^{-1} V_k: Eq.(3);
 *   - similarity criterion d(A,B) = ||I - A B^{-1}||_2: Eq.(5), and the
 *     entrywise l1 / Frobenius criteria of the remark after Eq.(4);
 *   - database construction: Algorithm 1 (tolerance) and Algorithm 2 with the
 *     variants and the boundary partitioning of Section 3.2;
 *   - use as the preconditioner of GMRES (Section 4), optionally as the damped
 *     smoothing step x <- x + omega M^{-1} r (Experiment 3).
 *
 * Conventions (every entry point):
 *   - Arrays named "device" must be device memory of the current HIP device
 *     (e.g. torch.Tensor.data_ptr() of a CUDA/HIP tensor); arrays named "host"
 *     are ordinary host memory.  A host pointer where device memory is
 *     required returns PR_ERR_HOST_POINTER.
 *   - The caller owns every array it passes.  pr_setup copies the matrix and
 *     the patch lists into memory owned by the handle, so the caller may free
 *     them afterwards.  pr_destroy frees everything the handle owns.
 *   - Indices are 0-based.  Matrices inside patches are dense row-major.
 *   - Return value: PR_OK (0), a positive warning, or a negative error code;
 *     pr_last_error() gives a message for the last failure on a handle.
 *   - pr_apply is asynchronous on the handle's stream; pr_setup and pr_solve
 *     synchronise it.  A handle is not thread-safe; distinct handles are
 *     independent.
 */
#ifndef PATCHRELAX_H
#define PATCHRELAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PR_OK                     0
#define PR_NOT_CONVERGED          1   /* solve stopped at max_iters; x holds the last iterate */
#define PR_ERR_INVALID_ARG       -1   /* null pointer, negative size, bad parameter value */
#define PR_ERR_HOST_POINTER      -2   /* host memory passed where device memory is required */
#define PR_ERR_DOF_OUT_OF_RANGE  -3   /* a patch lists a dof outside [0, n) */
#define PR_ERR_DUP_DOF_IN_PATCH  -4   /* a dof appears twice in one patch */
#define PR_ERR_UNCOVERED_DOF     -5   /* a dof lies in no patch: W undefined (Section 2) */
#define PR_ERR_SINGULAR_PATCH    -6   /* zero pivot while inverting a database matrix */
#define PR_ERR_NONFINITE         -7   /* NaN/Inf in a tile, right-hand side or solve */
#define PR_ERR_OOM               -8   /* device allocation failed */
#define PR_ERR_HIP               -9   /* other HIP runtime error (message kept) */
#define PR_ERR_UNSUPPORTED      -10   /* valid input outside what the library supports */
#define PR_ERR_BAD_CSR          -11   /* row_ptr not monotone, column out of range or unsorted */
#define PR_ERR_BAD_PATCH_PTR    -12   /* patch ptr not monotone or an empty patch */

/* ---- enumerations ------------------------------------------------------ */
enum pr_algo {
    PR_ALGO_FULL = 0,              /* every patch is its own database entry: Eq.(1) */
    PR_ALGO_TOLERANCE = 1,         /* Algorithm 1 */
    PR_ALGO_KMEANS_SPECTRAL = 2,   /* Algorithm 2: spectral distance, mean centres (Eq.(6)) */
    PR_ALGO_KMEANS_ENTRYWISE = 3,  /* Algorithm 2: l1 distance to the mean, mean centres */
    PR_ALGO_VARMIN = 4,            /* Algorithm 2: spectral distance, medoid centres */
    PR_ALGO_BOOTSTRAP = 5          /* Algorithm 1 then variance-minimising Algorithm 2 */
};
enum pr_criterion { PR_CRIT_SPECTRAL = 0, PR_CRIT_L1 = 1, PR_CRIT_FRO = 2 };
/* Arithmetic of the patch solves in the apply.  BF16 / FP16 / BF16X3 use
 * MFMA with FP32 accumulation; FP16 scales each database inverse and each
 * restricted residual by a power of two; BF16X3 splits both operands into a
 * BF16 high part and a BF16 remainder and sums the three leading products
 * (about 16 significant bits). */
enum pr_precision { PR_FP64 = 0, PR_FP32 = 1, PR_BF16 = 2, PR_FP16 = 3, PR_BF16X3 = 4 };
enum pr_apply_form { PR_FORM_AUTO = 0, PR_FORM_GENERAL = 1, PR_FORM_TILES = 2 };

/* ---- argument structs -------------------------------------------------- */

/* Global n x n matrix A in CSR form, all arrays device memory.
 * row_ptr int64[n+1] (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz);
 * col int32[nnz], strictly increasing within each row, in [0, n);
 * val double[nnz]. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
} pr_csr;

/* Patches (Section 2): patch k lists global dofs dofs[ptr[k] .. ptr[k+1]).
 * The list order is the local order of V_k.  ptr int64[n_p+1] and dofs
 * int32[ptr[n_p]] are device memory.  Each patch holds 1..32 distinct dofs
 * and every dof in [0, n) must lie in at least one patch. */
typedef struct {
    int64_t n_p;
    const int64_t* ptr;
    const int32_t* dofs;
} pr_patches;

/* Parameters; pr_params_default() fills every field. */
typedef struct {
    int32_t algo;            /* enum pr_algo (default PR_ALGO_FULL) */
    int32_t criterion;       /* enum pr_criterion for Algorithm 1 (default spectral) */
    double  eps;             /* Algorithm 1 tolerance, strict d < eps (default 1e-8) */
    int64_t m_target;        /* Algorithm 2 database size m_p */
    int32_t partition_bc;    /* Algorithm 2: cluster boundary groups separately (default 1) */
    int32_t kmeans_max_iter; /* Algorithm 2 pass limit (default 100) */
    uint64_t seed;           /* SplitMix64 seed of Algorithm 2's initial draw (default 5) */
    double  tie_rel;         /* relative argmin tie band (default 1e-9) */
    int32_t apply_precision; /* enum pr_precision of the patch solves (default FP64) */
    double  omega;           /* damping (default 1.0) */
    int32_t sweeps;          /* smoothing steps per preconditioner application (default 1) */
    int32_t gmres_restart;   /* GMRES restart length (default 30) */
    int64_t max_iters;       /* GMRES iteration limit (default 10000) */
    int32_t deterministic;   /* 1: scatter without floating-point atomics (default 0) */
    int32_t timing;          /* 1: pr_solve brackets its kernels with HIP events and
                                reports per-class device time in pr_solve_info; k > 1:
                                only the kernels of every k-th Arnoldi step (an event adds
                                a few microseconds between kernels) (default 0) */
    void*   stream;          /* hipStream_t for all work (NULL = default stream) */
    /* learned entry predictor for Algorithm 1 (pr_setup, PR_ALGO_TOLERANCE) */
    int32_t mlp;             /* 1: Algorithm 1 with predictions (default 0) */
    int32_t mlp_topk;        /* candidates tried per patch, 1..8 (default 4) */
    double  mlp_train_frac;  /* fraction of patches in the training set, (0, 1] (default 0.1) */
    int32_t mlp_epochs;      /* passes over the training set (default 60) */
    int32_t mlp_hidden;      /* width of both hidden layers, 1..1024 (default 64) */
    uint64_t mlp_seed;       /* SplitMix64 seed: sample, weights, shuffles (default 6) */
    double  mlp_lr;          /* Adam learning rate (default 3e-3) */
    int32_t mlp_batch;       /* minibatch rows (default 256) */
    int32_t mlp_precision;   /* PR_FP16 (MFMA, FP32 accumulate; default) or PR_FP32 */
    int32_t graph;           /* 1: pr_solve captures one restart cycle in a HIP graph and
                                replays it (ignored with timing != 0; default 0) */
    int32_t autotune;        /* 1: pr_setup times the apply's launch shapes and keeps the
                                fastest (default 0).  The choice is kept per process, keyed
                                on the device and the apply's shape (n, patches, entries,
                                groups, patch sizes, precision, scatter mode); a later setup
                                of the same shape reuses it without timing */
    int32_t apply_form;      /* PR_FORM_AUTO (default): when every patch has the same size
                                of at most 16 dofs and the database groups are long (at
                                most 1.25 work items per 16-patch tile), the MFMA apply
                                runs over fixed tiles of 16 grouped patches, otherwise over
                                work items of one database entry each; when no dof lies in
                                more than 8 patches the deterministic slot sum reads a
                                padded per-dof slot table;
                                PR_FORM_TILES: as AUTO, but fixed tiles (of 16 or 32
                                patches) whenever every patch has the same size of at most
                                32 dofs;
                                PR_FORM_GENERAL: work items per database entry and CSR slot
                                lists.  All three give the same bits */
    int32_t alg1_prune;      /* Algorithm 1: 1 (default) skips the pairs a certified bound
                                rules out (patches sorted by the Frobenius norm, or the l1
                                norm for the l1 criterion; a pair whose norms differ by more
                                than the criterion allows cannot match), which changes
                                neither phi nor the database; 0 evaluates every pair the
                                sequential algorithm compares, so crit_evals equals that
                                algorithm's comparison count and crit_pruned is 0 */
    int32_t alg1_match;      /* Algorithm 1 (PR_ALGO_TOLERANCE without mlp): 0 (default) maps a
                                patch to the first entry within eps, as printed; 1 maps it to
                                the closest of the entries within eps that exist when it is
                                visited (the variant of the remarks after Algorithm 1; the
                                database is the same).  Equal distances: entries with
                                d <= d_min (1 + tie_rel) + tie_rel s (s = 1 spectral, sum |A_i|
                                for l1, ||A_i||_F for Frobenius) tie and the lowest index wins */
    int32_t flexible;        /* pr_solve without systems: 1 keeps the preconditioned vectors
                                z_j = M v_j of a restart cycle and updates x += Z y (flexible
                                GMRES) instead of applying M to V y; the same iterates for an
                                exactly linear preconditioner, and no drift between the
                                residual estimate and the true residual when the apply rounds
                                its input to reduced precision; n x gmres_restart more
                                doubles (default 0) */
    int32_t orth;            /* pr_solve without systems, gmres_restart <= 31: 0 (default)
                                classical Gram-Schmidt with delayed reorthogonalisation
                                (every vector projected twice, the second projection folded
                                into the next step's pass: two passes over the basis per
                                Arnoldi step; the stopping test sees a column one step
                                later); 1 classical Gram-Schmidt whose second projection runs
                                when the first lost more than a factor sqrt(2) (three passes
                                when it runs).  Restarts above 31 take form 1 */
} pr_params;

/* Interpolation P0 from n_coarse coarse unknowns to the n_fine fine ones
 * (CSR, n_fine rows, column indices in [0, n_coarse), device arrays):
 * row_ptr int64[n_fine+1], col int32[nnz], val double[nnz]. */
typedef struct {
    int64_t n_fine;
    int64_t n_coarse;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
} pr_interp;

typedef struct pr_handle_s* pr_handle;

typedef struct {
    int64_t iters;           /* Arnoldi steps taken */
    int64_t cycles;          /* restart cycles */
    double  relres;          /* true ||b - A x||_2 / ||b||_2 at exit, FP64 */
    double  relres_est;      /* GMRES estimate at exit */
    int32_t status;          /* PR_OK or PR_NOT_CONVERGED or an error */
    int32_t reorth;          /* Arnoldi steps that took the second Gram-Schmidt projection
                                (selective reorthogonalisation; every step beyond 31 basis
                                vectors and every step of a batch solve counts) */
    double  seconds;         /* wall time of the last pr_solve */
    /* with params.timing != 0: device milliseconds and launch counts of the
     * preconditioner applications (zero fill + apply kernel), the sparse
     * matrix-vector products and the Gram-Schmidt orthogonalisation */
    double  apply_ms, spmv_ms, orth_ms;
    int64_t n_apply, n_spmv, n_orth;
    /* with a coarse space (pr_set_coarse) and params.timing != 0: device
     * milliseconds and count of the coarse terms P0 A0^{-1} R0 v (apply_ms
     * then covers the patch part alone) */
    double  coarse_ms;
    int64_t n_coarse;
} pr_solve_info;

typedef struct {
    int64_t n, nnz, n_p, m_p;
    int32_t max_ps, min_ps;
    int32_t n_groups;        /* distinct boundary keys */
    int32_t algo;
    int64_t crit_evals;      /* criterion evaluations made */
    int64_t crit_pruned;     /* pairs skipped by the certified norm bound */
    int64_t crit_exact;      /* evaluations that needed the exact singular value */
    int64_t alg1_rounds;     /* Algorithm 1 rounds: one entry per component and round, up
                                to 16 after the batched inversion (alg1_batch_inverted) */
    int64_t kmeans_iters;    /* Algorithm 2: most assignment passes of any group */
    int64_t empty_events;    /* Algorithm 2 empty clusters */
    int64_t n_items;         /* grouped apply work items */
    int64_t bytes_tiles, bytes_db, bytes_db_lowp, bytes_index;
    double  t_validate, t_extract, t_database, t_factor, t_group, t_total; /* seconds */
    int32_t apply_precision;
    int32_t apply_tile_p;    /* > 0: the MFMA apply runs over fixed tiles of patches of this
                                size (see apply_form); 0: over work items (n_items) */
    /* Algorithm 1 with predictions (params.mlp = 1) */
    int64_t mlp_train;       /* training patches */
    int64_t mlp_classes;     /* entries of the training database (network classes) */
    int64_t mlp_accepted;    /* patches matched by a predicted candidate */
    int64_t mlp_scanned;     /* patches matched by the in-order scan */
    int64_t mlp_fallback;    /* patches left to Algorithm 1 (matched nothing) */
    double  mlp_loss;        /* mean cross-entropy on the training set after training */
    double  mlp_train_acc;   /* top-1 accuracy on the training set */
    double  t_mlp_train;     /* seconds: features, training and the accuracy pass */
    /* apply launch shape (params.autotune = 1: the fastest measured; else 0 = defaults) */
    int32_t tune_threads;    /* threads per block of the patch kernel */
    int32_t tune_slot;       /* threads per block of the slot sum */
    int64_t tune_cap;        /* block cap of the patch kernel (0 = none) */
    double  t_autotune;      /* seconds spent timing shapes (inside t_total) */
    int64_t tune_tiles_per_wave;  /* fixed-tile MFMA kernel: tiles per wavefront (1 or 2;
                                     0 = default, which is 1) */
    int64_t tune_xcd_remap;  /* 1: fixed-tile kernel and padded slot sum give each XCD one
                                contiguous range of blocks (0 = launch order); 1 unless the
                                tuner found launch order faster */
    int64_t crit_refined;    /* spectral evaluations the cheap bracket left open and the
                                repeated-squaring bracket then decided or narrowed */
    /* the solve's copy of A: 64-row slices, each in diagonal form (values per
       distinct column offset, 8 bytes each) or column form (values and
       column indices, 12 bytes each), whichever stores fewer bytes */
    int64_t sell_slots;          /* stored values, padding included */
    int64_t sell_diag_slices;    /* slices in diagonal form */
    int64_t sell_diag_offsets;   /* their distinct offsets (stored columns) */
    int64_t sell_col_entries;    /* matrix entries in column-form slices */
    int64_t alg1_batch_inverted; /* 1: Algorithm 1 ran more than 14 rounds, then inverted its
                                    unresolved patches in one batch (same inverses, bit for
                                    bit) and opened up to 16 entries per component and round
                                    (same result and evaluation count; crit_refined and
                                    crit_exact then include speculative pair tests) */
    int64_t closest_evals;       /* alg1_match = 1: criterion evaluations of the closest-match
                                    pass (after Algorithm 1's own, which crit_evals counts) */
    int64_t closest_moved;       /* alg1_match = 1: patches whose entry differs from the first
                                    match */
    /* two-level combination (pr_set_coarse; zeros without it) */
    int64_t n_coarse;            /* coarse unknowns n0 */
    int64_t coarse_nnz;          /* entries of R0 A P0 kept */
    int64_t coarse_bandwidth;    /* largest |v - w| over its entries */
    int64_t coarse_block;        /* rows per block of the banded solve (0: dense inverse) */
    int64_t coarse_blocks;       /* blocks of the banded solve (1: dense inverse) */
    double  t_coarse;            /* seconds of pr_set_coarse */
    /* pr_setup_reuse with Algorithm 1 (zeros otherwise) */
    int64_t reuse_kept;          /* patches still within eps of their previous entry */
    int64_t reuse_rescanned;     /* patches placed on another entry by the in-order scan */
    int64_t reuse_appended;      /* entries appended for patches no entry matched */
    /* the solve's copy of A, third form: slices whose rows differ so much in
       length that the column form would pad them by more than 30 % (average
       row at least 32 entries) read their rows from the CSR copy */
    int64_t sell_csr_slices;     /* slices in that form */
    int64_t sell_csr_entries;    /* their matrix entries */
} pr_stats;

/* ---- entry points ------------------------------------------------------ */

/* Fill *p with the defaults listed at pr_params. */
void pr_params_default(pr_params* p);

/* Setup (Section 2, Section 3): validate, count covers and form W, extract
 * the dense patch matrices A_k, choose the database (algo) and phi, invert
 * the database matrices in FP64 (LU with partial pivoting semantics), group
 * patches by database entry and convert the inverses to apply_precision.
 * A, P: device arrays (copied).  *out receives a new handle on PR_OK.
 * Errors: INVALID_ARG, HOST_POINTER, BAD_CSR, BAD_PATCH_PTR,
 * DOF_OUT_OF_RANGE, DUP_DOF_IN_PATCH, UNCOVERED_DOF, SINGULAR_PATCH (the
 * patch id is in pr_last_error), NONFINITE, OOM, HIP, UNSUPPORTED (a patch
 * with more than 512 dofs, or an option listed below for patches above 32
 * dofs).  Synchronises the stream.
 *
 * Patches above 32 dofs (p_s = q (p+1)^d reaches 216 for the degree-5 cells
 * of Section 4, Experiment 3): when any patch has more than 32 dofs, every
 * patch of the handle takes kernels with a block of 256 threads per patch
 * and tiles, inverses and criterion products in device memory.  They support
 * PR_ALGO_FULL and PR_ALGO_TOLERANCE (first matching, all three criteria),
 * FP64 and FP32 applies, sweeps, the coarse space and pr_solve; Algorithm 2,
 * the learned predictor, closest matching, pr_setup_reuse, the 16-bit
 * applies, autotune and pr_set_systems return UNSUPPORTED.  Algorithm 1 opens
 * one entry per round there (alg1_rounds = m_p); the spectral criterion is
 * decided from a bracket on sigma_max^2 (column norms and the Frobenius norm,
 * then up to 40 squarings of E^T E), and crit_exact counts the pairs whose
 * bracket stayed open after them (d within about 1e-11 of eps), decided at
 * its geometric midpoint.  The FP32 apply multiplies FP32 inverses and FP32
 * residual values with FP64 accumulation.
 *
 * Clustering algorithms (Algorithm 2, Section 3.2): patches are grouped by
 * size and, with partition_bc = 1, by boundary key (PR_ALGO_BOOTSTRAP never
 * partitions); m_target clusters are apportioned to the groups by largest
 * remainders (at least one per group; INVALID_ARG unless groups <= m_target
 * <= n_p); the initial centres are drawn per group, groups in ascending
 * (size, key) order, by a partial Fisher-Yates shuffle of the group's
 * members in ascending patch id, driven by one SplitMix64 stream seeded with
 * `seed` (position i takes the member at i + (u mod (L - i))).
 * PR_ALGO_BOOTSTRAP starts from Algorithm 1's entries (criterion, eps).  A
 * pass assigns every patch of a still-active group to the centre of least
 * distance, keeping its current centre if that lies in the tie band
 * d <= d_min (1 + tie_rel) + tie_rel s (s = 1 for the spectral distance,
 * sum |A_i| for the l1 distance), else the lowest centre in it; a group stops
 * when no assignment changes or after kmeans_max_iter passes, otherwise its
 * centres are updated (entrywise mean in ascending member id, or for
 * VARMIN/BOOTSTRAP the member nearest the mean in Frobenius norm, lowest id
 * among squared distances <= min (1 + tie_rel) + tie_rel^2 ||mean||_F^2); an
 * empty cluster keeps its centre.  Singular centre:
 * SINGULAR_PATCH.  The criterion field is used only by Algorithm 1. */
int pr_setup(const pr_csr* A, const pr_patches* P, const pr_params* prm, pr_handle* out);

/* z = omega * M~^{-1} r (Eq.(3); Eq.(1) for PR_ALGO_FULL) for one smoothing
 * step.  r, z: device double[n], distinct.  Asynchronous on the stream. */
int pr_apply(pr_handle h, const double* r, double* z);

/* Solve A x = b by right-preconditioned GMRES(gmres_restart) from x = 0,
 * preconditioned by `sweeps` damped smoothing steps; stops when
 * ||b - A x||_2 <= tol ||b||_2 (true residual) or after max_iters.
 * b, x: device double[n].  Returns PR_OK, PR_NOT_CONVERGED or an error;
 * details via pr_get_solve_info.  Synchronises the stream. */
int pr_solve(pr_handle h, const double* b, double* x, double tol);

/* Two-level combination preconditioner (Eq.(2)): M_combo^{-1} = M~^{-1} +
 * P0 A0^{-1} R0 with R0 = P0^T and A0 = R0 A P0 solved directly (the first
 * two numerical experiments replace the AMG cycle by a direct solve of
 * R0 A P0).  P0 interpolates from a first-order discretisation on the same
 * mesh, e.g. by linear interpolation at the high-order nodes; it is copied.
 * The library forms R0 and A0 on the device (each entry of A0 summed in one
 * fixed order; entries at most 1e-13 of their row's largest magnitude, the
 * rounding residue of couplings that vanish exactly, are dropped) and
 * factors A0: for n0 <= 4096 its explicit inverse, otherwise block LU over
 * blocks of b rows (b = the bandwidth max |v - w|, rounded up to 32, at most
 * 4096), keeping the inverses of the Schur complements.  Neither step
 * pivots across 32 x 32 blocks, which suits symmetric positive definite A0.
 * Afterwards pr_apply gives z = omega M~^{-1} r + P0 A0^{-1} R0 r and
 * pr_solve uses the combination as its preconditioner (the coarse term is
 * added once per application, after the `sweeps` smoothing steps).  Once per
 * handle, before any pr_set_systems.  Errors: INVALID_ARG (sizes, a column
 * outside [0, n_coarse), a bad row_ptr, second call, a batch of systems),
 * HOST_POINTER, NONFINITE, UNSUPPORTED (a coarse row coupled to more than 256
 * coarse unknowns, a bandwidth beyond 4096), SINGULAR_PATCH (a zero pivot in
 * the coarse factorisation), OOM, HIP.  Synchronises the stream. */
int pr_set_coarse(pr_handle h, const pr_interp* P0);
/* Parity hook: A0 = R0 A P0 in CSR, host arrays.  Call with null arrays to
 * get *n0 and *nnz, then with row_ptr int64[n0+1], col int32[nnz] and val
 * double[nnz].  INVALID_ARG without a coarse space. */
int pr_get_coarse_matrix(pr_handle h, int64_t* n0, int64_t* nnz, int64_t* row_ptr, int32_t* col,
                         double* val);

/* Database reuse across a sequence of linear systems on the same patches
 * (time stepping, nonlinear iterations): the closing remarks of the third
 * numerical experiment suggest reusing the previous setup's database
 * assignments, and Section 3.2 initialising the clustering from the previous
 * step.
 *
 * pr_export_database writes the handle's patch map phi and entry patch ids
 * to the host buffer buf: 40 header bytes (magic "PRDB0001", n_p, m_p,
 * algo, criterion, eps), then int32 phi[n_p] and int32 reps[m_p]
 * (little-endian).  With buf NULL it only sets *bytes to the size; with a
 * buffer, *bytes must hold its capacity and receives the size written.
 * Errors: INVALID_ARG (null bytes, a buffer too small).
 *
 * pr_setup_reuse is pr_setup seeded with such a blob (host memory, `bytes`
 * long; the patches must be the same n_p, the matrix may differ):
 *  - PR_ALGO_TOLERANCE: the previous entries (patch ids, in their order) are
 *    the first entries, inverted from the current matrix.  Every other patch,
 *    in ascending id, keeps its previous entry when d < eps, else takes the
 *    first entry in append order with d < eps, else is appended (Algorithm 1
 *    on the patches that matched nothing).  Every patch then lies within eps
 *    of its entry, and entry numbers of kept patches do not change.
 *  - k-means variants: the passes start from the previous assignment; the
 *    centres start as its update (mean or medoid of the current matrices),
 *    so a system that barely changed converges in a pass or two.  m_target
 *    and the groups must match the blob, and every previous centre must
 *    keep a member.
 * Errors as pr_setup, plus INVALID_ARG for a malformed or mismatched blob,
 * PR_ALGO_FULL or PR_ALGO_BOOTSTRAP, mlp = 1 or closest matching. */
int pr_export_database(pr_handle h, void* buf, int64_t* bytes);
int pr_setup_reuse(const pr_csr* A, const pr_patches* P, const pr_params* prm, const void* db,
                   int64_t bytes, pr_handle* out);

int pr_get_solve_info(pr_handle h, pr_solve_info* info);
int pr_get_stats(pr_handle h, pr_stats* s);

/* Parity hooks (host outputs, synchronising):
 * phi: int32[n_p] database entry of each patch; reps: int32[m_p] patch whose
 * matrix is entry j (-1 for a cluster mean); *m_p: database size.  Any output
 * pointer may be NULL. */
int pr_get_assignment(pr_handle h, int32_t* phi, int32_t* reps, int64_t* m_p);
/* tile: double[p_k * p_k], the dense A_k of patch k, row-major. */
int pr_get_patch_tile(pr_handle h, int64_t k, double* tile);
/* W: double[n] (Section 2). */
int pr_get_weights(pr_handle h, double* W);
/* keys: uint32[n_p], bit a set iff local row a of A_k has exactly one
 * nonzero (boundary partitioning, Section 3.2).  For patches above 32 dofs
 * the key is the XOR over rows a with one nonzero of bit (a mod 32) (the
 * 32-bit fold of that row mask, equal to the mask up to 32 dofs). */
int pr_get_boundary_keys(pr_handle h, uint32_t* keys);
/* X: double[p_j * p_j], the FP64 inverse of database entry j, row-major. */
int pr_get_rep_inverse(pr_handle h, int64_t j, double* X);
/* B: double[p_j * p_j], the matrix of database entry j (a patch matrix, or
 * the cluster mean of Eq.(6)), row-major. */
int pr_get_entry_matrix(pr_handle h, int64_t j, double* B);
/* Algorithm 1 with predictions (params.mlp = 1): train receives the
 * stats.mlp_train training patch ids (ascending); cand receives
 * int32[n_p * mlp_topk], row i the predicted entries of patch i (indices
 * into the training database, most probable first; -1 for training patches
 * and unused slots).  Either pointer may be NULL.  INVALID_ARG without a
 * predictor. */
int pr_get_mlp_candidates(pr_handle h, int32_t* train, int32_t* cand);
/* The predictor's raw (not standardised) features: *F = 3 p_max + 1 and, if X
 * is not NULL, X: host float[n_p * F], row k for patch k (A_aa / m, then
 * sum_b |A_ab| / m, then the single-entry row bits, then log m, with
 * m = mean_a |A_aa|, slots beyond p_k zero).  INVALID_ARG without a predictor. */
int pr_get_mlp_features(pr_handle h, float* X, int32_t* F);

/* Independent systems (uneven batches): A is block diagonal with system s
 * on rows [system_ptr[s], system_ptr[s+1]) (host int64[n_sys+1], from 0 to
 * n, each range non-empty) and every patch lies inside one system.  Later
 * pr_solve calls run one right-preconditioned GMRES per system, each with
 * its own Krylov space and the stopping test ||b_s - A_s x_s|| <= tol ||b_s||;
 * converged systems are masked while the others continue, and every launch
 * serves all systems.  pr_solve_info then reports the largest iteration
 * count and relative residual over the systems.  Errors: INVALID_ARG (bad
 * ranges, a matrix entry or a patch across two systems).  Synchronises. */
int pr_set_systems(pr_handle h, const int64_t* system_ptr, int64_t n_sys);
/* Per-system results of the last pr_solve: iters host int64[n_sys], relres
 * host double[n_sys] (either may be NULL).  INVALID_ARG without systems. */
int pr_get_system_info(pr_handle h, int64_t* iters, double* relres);

/* Use another stream for later calls on h (NULL = default stream).  Waits
 * for the work queued on the old stream first. */
int pr_set_stream(pr_handle h, void* hip_stream);

/* Host-only validation of host arrays (no GPU needed): same checks and codes
 * as pr_setup performs on the device. */
int pr_validate_host(const pr_csr* A_host, const pr_patches* P_host);

/* Waits for the handle's stream and returns everything it owns.  Its device
 * buffers go to the device memory cache below, not back to the HIP runtime. */
void pr_destroy(pr_handle h);
const char* pr_status_string(int status);
const char* pr_last_error(pr_handle h);   /* h may be NULL: last global error */

/* ---- device memory cache ------------------------------------------------
 * Library bookkeeping, not part of the method.  Every device buffer a handle
 * owns is taken from a per-device cache of idle blocks and returned to it by
 * pr_destroy, so a sequence of setups on one device maps memory once (hipFree
 * synchronises the device and unmaps pages; a cached block costs neither).
 * Idle blocks stay allocated until evicted: by default at most one eighth of
 * the device's memory is kept idle per device (largest blocks are freed
 * first); an allocation that fails frees the idle blocks of its device and
 * tries once more.  A cached block is never shared by two live handles.
 * Thread-safe. */

/* Idle bytes kept per device from now on (0 disables caching, -1 restores
 * the default); frees idle blocks beyond it.  INVALID_ARG below -1. */
int pr_set_memory_cache_limit(int64_t bytes);
/* Frees every idle block on every device (e.g. before handing the memory to
 * another allocator).  Handles stay valid. */
int pr_release_cached_memory(void);
/* info: host int64[4] = {idle bytes, idle blocks, allocations served from
 * the cache, allocations that called hipMalloc} for `device` (-1: pinned
 * host blocks); zeros for a device never used.  INVALID_ARG for a null info
 * or a device below -1.  Needs no GPU. */
int pr_memory_cache_info(int32_t device, int64_t* info);

/* ---- standalone batched kernels (device arrays, asynchronous) ----------- */

/* Batched inverse of `count` dense p x p matrices (row-major, contiguous),
 * Gauss-Jordan elimination with partial pivoting in FP64, one wavefront per
 * matrix (the factorisation step of Section 4, Experiment 3).  A: device
 * double[count*p*p]; X: device double[count*p*p]; info: device
 * int32[count], 0 or the 1-based column of the first zero pivot.
 * 1 <= p <= 512; above 32 a block of 256 threads per matrix eliminates in
 * place in X with partial pivoting over the whole column. */
int pr_batch_inverse(int32_t p, int64_t count, const double* A, double* X, int32_t* info,
                     void* stream);

/* Batched criterion between A[i] and B[i] (Eq.(5) and the remark after
 * Eq.(4)): spectral d = ||I - A[i] X[i]||_2 with X[i] = B[i]^{-1} given
 * (largest singular value by cyclic Jacobi on E^T E), l1 sum|A - B|,
 * Frobenius ||A - B||_F.  A, B, X: device double[count*p*p] (B unused for
 * spectral, X unused otherwise; may be NULL then); d: device double[count]. */
int pr_batch_criterion(int32_t p, int64_t count, int32_t criterion, const double* A,
                       const double* B, const double* X, double* d, void* stream);

/* The learned entry predictor's network (the neural shortcut to building
 * the database that the closing remarks of Section 3.2 point to):
 * h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), logits = h2 W3 + b3, loss =
 * mean over rows of logsumexp(l) - l[y], the sum over the classes c with
 * class_key[c] == row_key[r] (all classes when both keys are NULL).
 * params, grads: device float[F*H + H + H*H + H + H*C + C], packed W1 (F x H,
 * row-major), b1, W2 (H x H), b2, W3 (H x C), b3.  X: device float[rows*F]
 * row-major; y: device int32[rows]; row_key: device int32[rows]; class_key:
 * device int32[C].  precision: PR_FP32 (FMA) or PR_FP16 (operands rounded
 * to FP16, MFMA, FP32 accumulation).  *loss: host double.  Synchronises
 * the stream.  Errors: INVALID_ARG (sizes, precision, a key missing),
 * HOST_POINTER, OOM. */
int pr_mlp_loss_grad(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C, const float* X,
                     const int32_t* y, const int32_t* row_key, const int32_t* class_key,
                     const float* params, float* grads, double* loss, void* stream);
/* Forward pass of the same network: logits (device float[rows*C], may be
 * NULL) and the k (0..8, at most C) allowed classes of largest logit per row,
 * largest first, lower index on ties (device int32[rows*k]; -1 when fewer
 * than k classes are allowed).  Synchronises the stream. */
int pr_mlp_predict(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C, const float* X,
                   const int32_t* row_key, const int32_t* class_key, const float* params, int32_t k,
                   float* logits, int32_t* topk, void* stream);

/* Size in bytes of the fixed device workspace of pr_mlp_predict_noalloc. */
#define PR_MLP_NOALLOC_SCRATCH_BYTES (32LL << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass and top-k as pr_mlp_predict, with the same arguments and the
 * same results, but it calls no hipMalloc, hipFree or other allocating
 * routine and does not synchronise (asynchronous on `stream`).  The hidden
 * activations, and the logits when `logits` is NULL, live in one fixed
 * device array of PR_MLP_NOALLOC_SCRATCH_BYTES that every device running
 * the library holds until the process ends; the first call on a device looks
 * up its address.  rows * (2 H + (logits ? 0 : C)) floats, each part rounded
 * up to 64 floats, must fit in it, else INVALID_ARG.  Every call on one
 * device shares that array: calls that overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.  Errors as for
 * pr_mlp_predict; a failed kernel launch gives HIP. */
int pr_mlp_predict_noalloc(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C,
                           const float* X, const int32_t* row_key, const int32_t* class_key,
                           const float* params, int32_t k, float* logits, int32_t* topk,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PATCHRELAX_H */
