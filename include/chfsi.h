/*
 * chfsi.h -- C ABI of the MI355X (gfx950) Chebyshev-filtered subspace
 * iteration library for real-space finite-difference Kohn-Sham DFT.
 *
 * The method: the Kohn-Sham Hamiltonian H = -1/2 Laplacian + V_eff + separable
 * Kleinman-Bylander projectors is discretised by a high-order (12th-order)
 * finite-difference stencil on a spherical real-space grid whose points are
 * stored along blockwise Hilbert space-filling curves; the lowest eigen-
 * subspace is tracked by Chebyshev-filtered subspace iteration (filter, then
 * Cholesky-QR orthonormalisation, then Rayleigh-Ritz), updated together with
 * the potential over the self-consistent-field (SCF) steps: four ChFSI
 * iterations in the first SCF step, one in each later step, until the
 * self-consistent residual error drops below 1e-4 Ry.
 * (Paper: the CheFSI paragraph, the sparse-product / space-filling-curve
 * paragraph, the computational-details paragraph and Table I.)
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: bohr and hartree.
 * Status: every call returns 0 (CHF_OK) or a negative CHF_E* code and never
 *   throws or aborts across the ABI; chf_last_error() returns a thread-local
 *   message for the last failing call on the calling thread.
 * Memory: all arrays named *_dev live in device memory and are owned by the
 *   caller; arrays named *_host live in host memory.  Handles own their
 *   internal tables until *_destroy.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *   asynchronous on that stream except where they return values in host
 *   memory, which synchronise the stream before returning.
 * Vector blocks: a block of nvec vectors is row-major [n_rows][ld] in the
 *   Hamiltonian's row order (see ham_export_ordering), vectors contiguous
 *   within a row, ld >= nvec.  Rows that hold no grid point (padding of the
 *   8^3 Hilbert blocks) must be zero on input and stay zero.  Orthonormality
 *   is Euclidean (X^T X = I, no h^3 factor).
 * Precision: CHF_F32 blocks are float, CHF_F64 blocks are double; the
 *   arithmetic of a call runs in that precision unless stated otherwise.
 * Errors: arguments are validated on the host before any launch (CHF_EINVAL);
 *   device failures map to CHF_EHIP.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHF_OK 0
#define CHF_EINVAL (-1)        /* bad argument (null, size, alignment, ld)        */
#define CHF_ENOMEM (-2)        /* device or host allocation failed               */
#define CHF_EHIP (-3)          /* HIP runtime / library error                    */
#define CHF_ENOTPD (-4)        /* Gram matrix not positive definite              */
#define CHF_ENOTCONV (-5)      /* iteration limit reached                        */
#define CHF_ENONFINITE (-6)    /* NaN or Inf met in an input or result           */
#define CHF_EUNSUPPORTED (-7)  /* valid request this build does not provide      */

typedef enum { CHF_F32 = 1, CHF_F64 = 2 } chf_dtype;

typedef enum { CHF_ORDER_HILBERT = 0, CHF_ORDER_LEX = 1 } chf_ordering;

typedef struct chf_ctx chf_ctx;
typedef struct chf_ham chf_ham;
typedef struct chf_scf chf_scf;

/* Thread-local text of the last error on this thread ("" if none). */
const char* chf_last_error(void);

/* ---------------------------------------------------------------------------
 * Context: rocBLAS / rocSOLVER handles and the M x M FP64 scratch used by the
 * dense subspace steps.  The scratch grows on demand (device allocation on
 * the first call that needs more) and is freed by chf_ctx_destroy.
 * ------------------------------------------------------------------------- */
int chf_ctx_create(int device, chf_ctx** out);
int chf_ctx_destroy(chf_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Hamiltonian construction (paper: the real-space finite-difference
 * discretisation, the spherical confined domain, the KB-form
 * pseudopotentials, and the blockwise Hilbert space-filling curves).
 *
 * Grid points: (i, j, k) * h with i^2 + j^2 + k^2 <= floor((radius / h)^2 +
 * 1e-9), origin at the centre atom.  ordering = CHF_ORDER_HILBERT: 8^3 blocks
 * counted from the bounding-box minimum corner, ordered by a 3-D Hilbert
 * index (Skilling's transpose algorithm, x the most significant axis), points
 * x-fastest inside a block, row = block slot * 512 + local index (padded).
 * ordering = CHF_ORDER_LEX: z-slowest, x-fastest over inside points, row =
 * rank (no padding).
 * ------------------------------------------------------------------------- */
typedef struct {
    double h;          /* grid spacing (bohr), > 0                                 */
    double radius;     /* domain radius (bohr), > h                                */
    int ordering;      /* chf_ordering                                             */
    int keep_nbr;      /* nonzero: keep the per-row 36-neighbour table on device   */
                       /* (always kept for CHF_ORDER_LEX)                          */
    int dtypes;        /* bit mask of precisions to prepare: 1 = F32, 2 = F64      */
} chf_grid_desc;

typedef struct {
    int n_atoms;
    const double* pos_host;      /* [n_atoms][3] bohr                                */
    const int* species_host;     /* [n_atoms]; 0 = Si (KB projectors), 1 = H         */
} chf_atoms;

/* Model pseudopotential: V_loc(r) = -sum_a Z_a erf(|r - R_a| / r_loc_a) /
 * |r - R_a| (finite r -> 0 limit), one s and one p Gaussian projector per Si
 * p_l(r) = N_l r^l exp(-r^2 / (2 r_c^2)) (int p_l^2 r^2 dr = 1) times real
 * harmonics, cut at |r - R_a| <= r_cut, KB energies h_s and h_p. */
typedef struct {
    double z_si, z_h;            /* ionic charges                                    */
    double r_loc_si, r_loc_h;    /* erf widths of the local part                     */
    double r_c, r_cut;           /* projector width and cutoff radius                */
    double h_s, h_p;             /* KB energies (Ha)                                 */
} chf_pp;

/* Builds the grid, the ordering, the neighbour and block tables, the
 * projector tables (host), uploads them, and computes V_loc on the device in
 * FP64; V_eff starts equal to V_loc.  The handle is bound to the device that
 * is current at the call.  Errors: CHF_EINVAL (null argument, h or radius not
 * positive and finite, radius <= h or radius / h >= 4000, bad ordering or
 * dtypes mask, species other than 0 and 1, non-finite position, pseudopotential
 * radii not positive, more than 2^31 rows or projector pairs), CHF_ENOMEM
 * (host or device allocation), CHF_EHIP; on error *out is NULL (when out is
 * not) and nothing stays allocated. */
int ham_build(const chf_grid_desc* grid, const chf_atoms* atoms, const chf_pp* pp,
              void* stream, chf_ham** out);

/* Host-only construction of the same ordering (no device needed): fills
 * *n_points and *n_rows; when the arrays are non-NULL also ijk_host
 * [n_points][3], row_of_rank_host [n_points] and nbr_host [n_points][36]
 * (neighbour ranks, -1 outside) -- call once with NULL arrays to size them. */
int chf_ordering_host(const chf_grid_desc* grid, int64_t* n_points, int64_t* n_rows, int32_t* ijk_host,
                      int64_t* row_of_rank_host, int32_t* nbr_host);

/* Host-only projector tables: *n_pairs (point, Si) pairs; when non-NULL,
 * sup_off_host [n_Si + 1] offsets, sup_rank_host [n_pairs] point ranks
 * (ascending within an atom), sup_beta_host [n_pairs][4] (s, px, py, pz)
 * projector values without the h^3 or KB-energy factors. */
int chf_projectors_host(const chf_grid_desc* grid, const chf_atoms* atoms, const chf_pp* pp, int64_t* n_pairs,
                        int64_t* sup_off_host, int32_t* sup_rank_host, double* sup_beta_host);
int ham_destroy(chf_ham* ham);

/* n_points: grid points inside the sphere; n_rows: rows of a vector block
 * (>= n_points); n_blocks: occupied 8^3 blocks (0 for CHF_ORDER_LEX);
 * n_proj: KB projector atoms; n_pairs: (point, projector atom) pairs. */
int ham_info(const chf_ham* ham, int64_t* n_points, int64_t* n_rows, int64_t* n_blocks,
             int64_t* n_proj, int64_t* n_pairs);

/* Host copies of the ordering, by rank (curve order of the points):
 * ijk_host [n_points][3] integer coordinates; row_of_rank_host [n_points];
 * nbr_host [n_points][36] neighbour ranks or -1 (offsets axis-major x, y, z,
 * each -6..-1 then +1..+6).  Any pointer may be NULL. */
int ham_export_ordering(const chf_ham* ham, int32_t* ijk_host, int64_t* row_of_rank_host,
                        int32_t* nbr_host);

/* V_loc on the rows (FP64, [n_rows], padding rows 0) into vloc_dev. */
int ham_get_vloc(const chf_ham* ham, double* vloc_dev, void* stream);

/* Sets V_eff from veff_dev (FP64 [n_rows]); padding rows are ignored.  FP32
 * copies are derived on the device.  Returns CHF_ENONFINITE (and leaves the
 * previous V_eff) if any inside value is NaN or Inf. */
int ham_set_veff(chf_ham* ham, const double* veff_dev, void* stream);

/* Y = H X for nvec vectors (paper: the sparse matrix-vector products on which
 * ChFSI's efficiency rests).  X and Y must not overlap.  Uses the handle's
 * KB-coefficient scratch (grown on demand). */
int ham_apply(chf_ham* ham, chf_dtype dtype, const void* X_dev, int64_t ldx, void* Y_dev,
              int64_t ldy, int nvec, void* stream);

/* Degree-m scaled Chebyshev filter (paper: the CheFSI paragraph; the Zhou-Saad
 * form): X <- T_m((H - c) / e) X / T_m((a0 - c) / e), e = (b - a) / 2,
 * c = (b + a) / 2, evaluated by the three-term recurrence in place over X and
 * work (work: [n_rows][ldw], same dtype, disjoint from X, ldw >= 1; its
 * contents on return are unspecified).  The vectors are independent, so a
 * work block narrower than nvec is used column block by column block
 * (min(nvec, ldw) vectors, rounded down to a multiple of 64 when ldw < nvec
 * and ldw >= 64, else to a multiple of 4 when ldw >= 4).  The tiled kernel of
 * the Hilbert layout takes blocks whose width and leading dimensions are
 * multiples of 2 (FP32) and 8-byte aligned; other blocks, such as the 1- to
 * 3-column blocks of a work block with ldw < 4, take the neighbour-table
 * kernel, which needs a handle built with keep_nbr.  Requires a < b and
 * a0 < a; 1 <= degree <= 1000.  Errors: CHF_EINVAL (null block, ld < nvec,
 * bounds, X and work overlapping), CHF_EUNSUPPORTED (a block only the
 * neighbour-table kernel takes, on a handle without the table), CHF_EHIP. */
int chebyshev_filter(chf_ham* ham, chf_dtype dtype, void* X_dev, int64_t ldx, int nvec, int degree,
                     double a, double b, double a0, void* work_dev, int64_t ldw, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as chebyshev_filter, same arguments, results and errors, except
 * that it makes no device allocation and records no kernel timers.  The KB
 * coefficients it rewrites every degree step live in a fixed 64 MiB device
 * array that the library holds on each device it runs on until the process
 * ends (set up by the first ham_build on that device), instead of in the
 * handle's scratch.  The block is filtered in column blocks of
 * min(nvec, ldw, 64 MiB / (4 n_proj sizeof(element))) vectors, rounded down
 * to a multiple of 64 (or of 4) when fewer than nvec.  Limit: CHF_EINVAL if
 * the coefficients of one vector, 4 n_proj elements, exceed 64 MiB (more
 * than 4,194,304 FP32 or 2,097,152 FP64 projector atoms).  Every call on a
 * device shares that device's array: calls that overlap on one device (on
 * different streams or threads) race and must be serialised by the caller.
 * Nothing in the array needs to start at zero: each degree step overwrites
 * the coefficients it reads. */
int chebyshev_filter_noalloc(chf_ham* ham, chf_dtype dtype, void* X_dev, int64_t ldx, int nvec, int degree,
                             double a, double b, double a0, void* work_dev, int64_t ldw, void* stream);

/* The same operator and filter forced onto the neighbour-table kernel (needs
 * keep_nbr): a layout-independent second device path used to cross-check the
 * Hilbert-tiled kernel. */
int chf_ham_apply_generic(chf_ham* ham, chf_dtype dtype, const void* X_dev, int64_t ldx, void* Y_dev,
                          int64_t ldy, int nvec, void* stream);
int chf_filter_generic(chf_ham* ham, chf_dtype dtype, void* X_dev, int64_t ldx, int nvec, int degree,
                       double a, double b, double a0, void* work_dev, int64_t ldw, void* stream);

/* Kernel timing (instrumentation): while enabled, HIP events are recorded on
 * the launch stream around every H X launch (slot 0) and every KB-gather
 * launch (slot 1).  chf_timer(1) clears and enables, chf_timer(0) disables;
 * chf_timer_read synchronises the device and returns per slot the summed
 * milliseconds (ms_host[2]) and the launch counts (launches_host[2]).  The
 * timer is process-wide and thread-safe; its events belong to the device
 * current at each launch, so read it with that device current. */
int chf_timer(int enable);
int chf_timer_read(double* ms_host, int64_t* launches_host);

/* k-step Lanczos (FP64) from v0_dev ([n_rows], padding zero): out3_host =
 * {b = largest Ritz value + residual norm, smallest Ritz value, largest Ritz
 * value}.  Upper bound of the spectrum used by the filter.  2 <= k <= 64. */
int lanczos_bound(chf_ham* ham, chf_ctx* ctx, const double* v0_dev, int k, double* out3_host,
                  void* stream);

/* S = A^T B for row-major blocks A [n_rows][lda] (m columns) and B [n_rows][ldb]
 * (n columns): products of row slices (at most 8192 rows each, whatever the
 * width, so that no sum in the block precision runs over more rows) accumulated
 * on MFMA in the block precision (rocBLAS), the slice partials added in FP64 in
 * slice order.  S_dev is FP64 row-major [m][lds].  With A == B and m == n the
 * upper triangle is summed and mirrored, so S is exactly symmetric. */
int gram(chf_ctx* ctx, chf_dtype dtype, const void* A_dev, int64_t lda, const void* B_dev,
         int64_t ldb, int64_t n_rows, int m, int n, double* S_dev, int64_t lds, void* stream);

/* Workspace.  The library keeps device scratch on the handles (KB
 * coefficients on the Hamiltonian; M x M matrices, Gram partials, Lanczos
 * vectors and reduction partials on the context) and grows it on first use
 * at a larger size.  For an operation at nvec vectors of dtype on the
 * Hamiltonian's grid, chf_workspace_bytes reports the scratch it grows to on
 * each handle (ldw: the Rayleigh-Ritz work leading dimension, ignored
 * otherwise); chf_reserve grows it now, so later calls of that operation at
 * the same or smaller sizes make no device allocation in this library
 * (rocBLAS / rocSOLVER keep their own workspace on the context's handle,
 * grown by them on first use).  Operations: */
enum {
    CHF_WS_FILTER = 0,          /* ham_apply, chebyshev_filter */
    CHF_WS_ORTHONORMALIZE = 1,  /* orthonormalize over the grid's n_rows */
    CHF_WS_RAYLEIGH_RITZ = 2,   /* rayleigh_ritz */
    CHF_WS_LANCZOS = 3          /* lanczos_bound */
};
int chf_workspace_bytes(const chf_ham* ham, int op, chf_dtype dtype, int nvec, int64_t ldw, int64_t* ham_bytes,
                        int64_t* ctx_bytes);
/* ctx may be NULL for CHF_WS_FILTER.  CHF_ENOMEM if the device is full. */
int chf_reserve(chf_ham* ham, chf_ctx* ctx, int op, chf_dtype dtype, int nvec, int64_t ldw);
/* Device allocations made by the library so far in this process (a counter
 * for checking that a sequence of calls allocates nothing). */
int64_t chf_device_allocations(void);

/* Cholesky-QR (paper: the subspace orthonormalisation of ChFSI, CheFSI
 * paragraph): S = X^T X (gram), S = R^T R in FP64, X <- X R^{-1} (the
 * update in the block precision), in place on X [n_rows][ldx] (nvec columns,
 * n_rows >= nvec).  gram_dtype: precision of the Gram products -- CHF_F64
 * for an FP64 block; for an FP32 block CHF_F32 (FP32 MFMA products within
 * row slices, the slices summed in FP64) or CHF_F64 (FP64 products of the
 * widened block).  FP64 blocks take one pass; FP32 blocks take two (the
 * second on the result of the first, CholQR2), which gives the same Q as one
 * exact pass and removes the orthogonality loss of about kappa^2 u_32 that
 * one FP32 pass leaves on an ill-conditioned (filtered) block.
 * Breakdown of the first pass: the factorisation fails, or a pivot R_ii^2
 * falls below a fraction of column i's squared norm (1e-13 with an FP64
 * Gram, 1e-5 with an FP32 Gram): the column is numerically dependent on the
 * ones before it.  Then an FP32 block with an FP32 Gram is redone with an
 * FP64 Gram, and if that (or an FP64 block's pass) breaks down too, a
 * shifted Cholesky-QR (shift 1e-14 (FP64) / 1e-6 (FP32) of the mean
 * diagonal) is followed by a plain pass.  *fallbacks (may be NULL) receives
 * the number of retries.  Errors: CHF_EINVAL (null block, nvec < 1, ldx <
 * nvec, n_rows < nvec, n_rows or ldx >= 2^31, a gram_dtype other than
 * CHF_F32 / CHF_F64, an FP64 block with an FP32 Gram), CHF_ENOTPD (the
 * shifted pass breaks down too; X then holds the last successful pass),
 * CHF_EHIP. */
int orthonormalize(chf_ctx* ctx, chf_dtype dtype, void* X_dev, int64_t ldx, int64_t n_rows, int nvec,
                   chf_dtype gram_dtype, int* fallbacks, void* stream);

/* Rayleigh-Ritz (paper: the CheFSI paragraph): W = H X in column blocks of
 * min(nvec, ldw) vectors through the work block ([n_rows][ldw], ldw >= 1,
 * same dtype as X, disjoint from it), Hs = X^T W symmetrised (FP64),
 * Hs = Q diag(eig) Q^T (FP64), X <- X Q in row panels of n_rows ldw / nvec
 * rows, in place (the work block holds one panel at a time; Q rounded to
 * FP32 for an FP32 block).  eig_host [nvec] ascending.  So the work block
 * can be much narrower than X: at 7552 FP64 states a 256-wide work block is
 * 1/30 of X.  Errors: CHF_EINVAL (null argument, ldx < nvec, ldw < 1, X and
 * work overlapping, nvec above the grid's point count, a handle without this
 * dtype), CHF_ENOTCONV (eigensolver), CHF_ENONFINITE (a Ritz value is NaN or
 * Inf; X is then unchanged). */
int rayleigh_ritz(chf_ham* ham, chf_ctx* ctx, chf_dtype dtype, void* X_dev, int64_t ldx, int nvec,
                  double* eig_host, void* work_dev, int64_t ldw, void* stream);

/* ---------------------------------------------------------------------------
 * SCF pieces (paper: Kohn-Sham DFT with LDA in the Perdew-Zunger form, SRE
 * convergence criterion, the 4-then-1 ChFSI schedule).  All FP64.
 * ------------------------------------------------------------------------- */

/* rho[row] = sum_{i < n_occ} 2 X[row][i]^2 / h^3 (closed shell). */
int chf_density(chf_ham* ham, chf_dtype dtype, const void* X_dev, int64_t ldx, int n_occ,
                double* rho_dev, void* stream);

/* Hartree potential: -L V = 4 pi rho on the inside points with the same
 * 12th-order stencil; stencil points outside the sphere take the l <= 4
 * multipole expansion of rho about the origin.  CG warm-started from vh_dev,
 * stops at ||r|| / ||b|| < rtol; *iters_host (may be NULL) receives the count.
 * CHF_ENOTCONV after max_iter iterations. */
int chf_hartree(chf_ham* ham, chf_ctx* ctx, const double* rho_dev, double* vh_dev, double rtol,
                int max_iter, int* iters_host, void* stream);

/* PZ81 unpolarised LDA: eps_xc and v_xc per row (0 where rho < 1e-14). */
int chf_lda(chf_ham* ham, const double* rho_dev, double* exc_dev, double* vxc_dev, void* stream);

/* Initial density: superposition of Gaussian atoms Z (alpha / pi)^(3/2)
 * exp(-alpha r^2) (Z = 4 for Si, 1 for H; exponents per species), rescaled so
 * that h^3 sum rho = n_electrons.  rho_dev [n_rows] FP64 (padding 0). */
int chf_sad_density(chf_ham* ham, const chf_atoms* atoms, double alpha_si, double alpha_h, int n_electrons,
                    double* rho_dev, void* stream);

/* Clamps rho_dev (FP64 [n_rows]) at zero and rescales it to h^3 sum rho =
 * n_electrons (used on a learned start density). */
int chf_density_fix(chf_ham* ham, double* rho_dev, int n_electrons, void* stream);

/* Ion-ion energy sum_{a < b} Z_a Z_b / |R_a - R_b| (host, Ha). */
int chf_ion_energy(const chf_atoms* atoms, const chf_pp* pp, double* out_host);

typedef struct {
    int n_electrons;      /* closed shell: n_electrons / 2 occupied states            */
    int nvec;             /* states tracked (columns of X)                            */
    int degree;           /* Chebyshev degree                                         */
    int first_iters;      /* ChFSI iterations in the first SCF step (paper: 4)        */
    int later_iters;      /* ChFSI iterations in each later step (paper: 1)           */
    int lanczos_k;        /* Lanczos steps for the upper bound                        */
    int filter_dtype;     /* chf_dtype of the filter (H X recurrences)               */
    int gram_dtype;       /* chf_dtype of the Gram products and X updates             */
    int mix_history;      /* Anderson history length                                  */
    double mix_beta;      /* Anderson mixing parameter                                */
    double cg_rtol;       /* Poisson CG relative tolerance                            */
    double e_ion;         /* ion-ion energy sum_{a<b} Z_a Z_b / R_ab (Ha)             */
} chf_scf_params;

typedef struct {
    int step;             /* 1-based SCF step just completed                         */
    int chfsi_iters;      /* ChFSI iterations done in it                             */
    int cg_iters;         /* Poisson CG iterations (both solves)                     */
    int chol_fallbacks;   /* Cholesky-QR fallbacks taken                             */
    double sre_ry;        /* self-consistent residual error (Ry)                     */
    double energy;        /* Harris-Foulkes total energy at rho_in (Ha)              */
    double band_energy;   /* sum f_i eps_i (Ha)                                      */
    double homo, lumo;    /* Ha                                                      */
    double bound_a, bound_b, bound_a0;  /* filter bounds used in the last iteration  */
} chf_scf_report;

/* SCF state: owns rho_in, V_H, the Anderson history and the filter bounds;
 * X and the work block stay caller-owned.  rho0_dev ([n_rows]) is the
 * initial density, v_lanczos_dev ([n_rows]) the fixed Lanczos start vector.
 * CHF_EINVAL for inconsistent parameters: an odd electron count, nvec not
 * above the occupied count or above the grid's point count, a bad schedule,
 * mixing, tolerance or dtype, an FP64 filter with an FP32 Gram, a handle
 * without FP64 or without the filter's dtype. */
int chf_scf_create(chf_ham* ham, chf_ctx* ctx, const chf_scf_params* params, const double* rho0_dev,
                   const double* v_lanczos_dev, chf_scf** out);
int chf_scf_destroy(chf_scf* scf);

/* One SCF step (paper: the CheFSI paragraph, where the subspace is improved
 * together with the potentials from one SCF iteration to the next, and the
 * computational-details paragraph: LDA-PZ, four ChFSI iterations in the first
 * step and one in each later step, SRE stopping criterion): V_eff from rho_in,
 * Lanczos bound, ChFSI iterations on X (filter, Cholesky-QR, Rayleigh-Ritz),
 * rho_out (scaled to hold the n_electrons electrons: h^3 sum rho_out = N_e,
 * which orthonormal FP64 columns give to rounding; FP32 columns only up to
 * the accumulation error of their Gram products), SRE, Harris-Foulkes
 * energy, Anderson mixing of rho_in; CHF_ENONFINITE if rho_out vanishes.  eig_host
 * (may be NULL) receives the nvec Ritz values.  X: [n_rows][ldx] in
 * filter_dtype, caller-owned and updated in place; work: [n_rows][ldw],
 * ldw >= 1 (the filter and Rayleigh-Ritz work in column blocks of
 * min(nvec, ldw) vectors and Rayleigh-Ritz rotates X in row panels, so a
 * narrow work block suffices), X and work disjoint.  Errors: CHF_EINVAL
 * (null argument, ldx < nvec, ldw < 1, X and work overlapping), CHF_ENONFINITE
 * (NaN or Inf in V_eff, singular Anderson history), CHF_ENOTCONV (Poisson CG
 * short of cg_rtol); errors of the filter, Cholesky-QR and Rayleigh-Ritz calls
 * it makes pass through unchanged. */
int scf_step(chf_scf* scf, void* X_dev, int64_t ldx, void* work_dev, int64_t ldw,
             chf_scf_report* report, double* eig_host);

/* Checkpoint access: copy rho_in / V_H ([n_rows] FP64) out of or into the
 * state (device to device, on the SCF's stream). */
int chf_scf_get_fields(chf_scf* scf, double* rho_in_dev, double* vh_dev);

/* Checkpoint / resume of the SCF state kept by the handle (the paper's runs
 * last days; a resumed run continues where the saved one stopped): step
 * counter, filter bounds, rho_in, V_H and the Anderson history.  The caller
 * owns X and saves it alongside.  chf_scf_state_size gives the length in
 * doubles (it grows with the history, up to 8 + (2 + 2 mix_history) n_rows);
 * chf_scf_save copies the state into state_host and synchronises;
 * chf_scf_load restores a state saved from an SCF of the same grid and
 * mixing history (CHF_EINVAL on a version, grid, history or size mismatch).
 * Resuming and stepping reproduces the uninterrupted run bit for bit. */
int chf_scf_state_size(const chf_scf* scf, int64_t* n_doubles);
int chf_scf_save(chf_scf* scf, double* state_host);
int chf_scf_load(chf_scf* scf, const double* state_host, int64_t n_doubles);

/* ---------------------------------------------------------------------------
 * Learned initial density: a 3-D U-Net (4 levels, `channels` channels, two
 * 3^3 conv + SiLU per level, stride-2 conv down, nearest upsample + 3^3 conv
 * up, skip concatenation, final 1^3 conv) mapping a scaled superposition-of-
 * atoms density on an S^3 patch to a scaled correction.  BF16 MFMA
 * convolutions with FP32 accumulation; FP32 master weights and Adam state.
 * Not in the paper: the method's extension that starts the SCF from a
 * corrected density; the plain superposition start remains the fallback.
 * ------------------------------------------------------------------------- */
typedef struct dnet dnet;

/* He-normal initialisation from `seed`; the output layer starts at zero. */
int dnet_create(int channels, uint64_t seed, dnet** out);
int dnet_destroy(dnet* net);
/* Number of FP32 master parameters (padded layout, see dnet_layer_info). */
int dnet_param_count(const dnet* net, int64_t* n);
/* Layer `layer` (0..20, in the order c1a c1b d1 c2a c2b d2 c3a c3b d3 c4a c4b
 * u3 c5a c5b u2 c6a c6b u1 c7a c7b out): info6 = {c_in, c_out, c_in padded,
 * c_out padded, kernel edge, stride}; offsets2 = {weight offset, bias
 * offset}.  Weights are [c_out padded][tap][c_in padded], tap = (dz*3+dy)*3+dx. */
int dnet_layer_info(const dnet* net, int layer, int* info6, int64_t* offsets2);
/* Host only: output edge of each of the 21 layers for patch edge S. */
int dnet_plan(int S, int* edges_host);
int dnet_get_params(const dnet* net, float* host);
int dnet_set_params(dnet* net, const float* host);
int dnet_get_grads(const dnet* net, float* host);
/* y_dev [S^3] = net(x_dev [S^3]) (x-fastest); keeps the activations for
 * dnet_backward.  S a multiple of 8 in [8, 512]. */
int dnet_forward(dnet* net, const float* x_dev, int S, float* y_dev, void* stream);
/* Accumulates parameter gradients of the last forward for dL/dy = dy_dev. */
int dnet_backward(dnet* net, const float* dy_dev, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected; step >= 1),
 * then clears the gradients. */
int dnet_adam(dnet* net, float lr, int step, void* stream);
/* Mean squared error of y against t (n values) into *loss_host, and
 * dL/dy = 2 (y - t) / n into dy_dev (may be NULL). */
int dnet_mse(dnet* net, const float* y_dev, const float* t_dev, int64_t n, double* loss_host, float* dy_dev,
             void* stream);
/* patch [S^3] = box [D^3] read at offset (ox, oy, oz) under cubic symmetry
 * sym in [0, 48) (axis permutation sym / 8, mirrored axes bits sym % 8);
 * cells outside the box read 0. */
int dnet_crop(const float* box_dev, int D, int S, int ox, int oy, int oz, int sym, float* patch_dev, void* stream);

/* out [D^3] = box - G_sigma * box: the box minus its blur by a separable
 * Gaussian of width sigma (cells), truncated at ceil(3 sigma) and
 * normalised, with zero values outside the box (x fastest).  Removes the
 * long-wavelength part of a predicted density correction, where the
 * network's errors concentrate.  work_dev: 2 D^3 floats of scratch; out may
 * alias neither box nor work.  Synchronises the stream. */
int dnet_highpass(const float* box_dev, int D, double sigma, float* out_dev, float* work_dev, void* stream);

/* Grid rows <-> cubic box of edge D (x-fastest) holding grid point (i, j, k)
 * at (i + off, j + off, k + off): box = scale * (rows - base_rows), the
 * difference taken in FP64 (base_rows_dev may be NULL: 0; cells without a
 * grid point 0); rows_out = base_rows + box / scale on inside rows (padding
 * 0; base_rows_dev may be NULL). */
int chf_rows_to_box(chf_ham* ham, const double* rows_dev, const double* base_rows_dev, double scale, float* box_dev,
                    int D, int off, void* stream);
int chf_box_to_rows(chf_ham* ham, const float* box_dev, int D, int off, double scale, const double* base_rows_dev,
                    double* rows_out_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CHFSI_H */
