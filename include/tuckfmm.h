/*
 * tuckfmm.h -- C ABI of an MI355X (gfx950) library for the aggregation and
 * disaggregation stages of the fast multipole method computed directly in Tucker
 * format, after C. Qian, M. Wang, A. C. Yucel, "Compression of Far-Fields in the
 * Fast Multipole Method via Tucker Decomposition" (arXiv 2103.05822).
 *
 * Notation (paper, Section II): a group is a non-empty FMM box B_v holding n_beta
 * RWG basis functions; the far-field (aggregation) matrix of a group and
 * polarisation alpha in {theta, phi} is A^alpha (N_dir x n_beta) with entries
 * P^{alpha,+}_{n,i} of eq. (4); N_dir = n_theta * n_phi plane-wave directions.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Complex numbers are interleaved (re, im).  "complex128" = two doubles,
 *    "complex64" = two floats.
 *  - Basis functions are numbered in group order: group g owns rows
 *    offsets[g] .. offsets[g+1]-1.  Direction index i = i_theta * n_phi + i_phi.
 *  - Dense far-field:  [N][2][n_theta][n_phi]   (polarisation 0 = theta, 1 = phi).
 *  - Vectors carry the right-hand-side index innermost:
 *        x, V : [N][nrhs]          F, G : [n_groups][2][N_dir][nrhs].
 *  - Tucker factors exchanged through the ABI use the paper's shapes, row-major:
 *        core [r_theta][r_phi][r_beta], U^theta [n_theta][r_theta],
 *        U^phi [n_phi][r_phi], U^beta [n_beta][r_beta]            (eq. (6)).
 *  - "device" pointers are HIP device memory of the current device, owned by the
 *    caller; "host" pointers are ordinary host memory, owned by the caller.
 *  - Compute calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*, NULL = default stream).  Outputs are overwritten, never accumulated.
 *  - Every call validates its arguments on the host before launching anything;
 *    on failure it returns a negative fmm_status and fmm_last_error() describes
 *    the problem.  Kernel faults surface as FMM_ERR_DEVICE at a later call.
 *    No call throws or aborts.
 */
#ifndef TUCKFMM_H
#define TUCKFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMM_OK = 0,
  FMM_ERR_ARG = -1,          /* null pointer, bad enum, value out of range      */
  FMM_ERR_SHAPE = -2,        /* inconsistent sizes, ranks or offsets             */
  FMM_ERR_SIZE = -3,         /* caller buffer too small                          */
  FMM_ERR_DEVICE = -4,       /* no usable GPU, or a HIP runtime error            */
  FMM_ERR_NUMERIC = -5,      /* NaN/Inf input or eigensolver failure             */
  FMM_ERR_UNSUPPORTED = -6,  /* precision or shape not supported by this build   */
  FMM_ERR_STATE = -7,        /* call order violated (e.g. compute before upload) */
  FMM_ERR_IO = -8            /* file missing, unreadable, truncated or corrupt   */
} fmm_status;

/* Storage / arithmetic precision of a compute path.
 *   FMM_C128   complex128 factors, FP64 arithmetic; x, F, G, V are complex128.
 *   FMM_C64    complex64 factors, FP32 arithmetic; x, F, G, V are complex64.
 *   FMM_BF16X2 complex64 factors and vectors; the products run on the bf16 matrix
 *              cores: every FP32 operand is split on chip into two bf16 pieces
 *              (hi + lo) and each product accumulates hi*hi + hi*lo + lo*hi in FP32
 *              (relative error of a product about 2^-16).  Needs an even nrhs.
 *   FMM_BF16X3 as FMM_BF16X2 with three pieces (hi + mid + lo) and the six products
 *              down to order 2^-16 (FP32-level error).  Needs an even nrhs.
 *
 * Kernels.  The streaming kernels run one workgroup per (group, polarisation,
 * right-hand side) and stream the factors from HBM once per right-hand side; they take
 * 64, 128, 256 or 512 threads by the mean item size, or as tuned (the environment
 * variable TUCKFMM_STREAM_THREADS, read at upload, fixes the default).  Untuned,
 * FMM_C128 and FMM_C64 run them for an odd nrhs and the matrix-core products (FP64
 * and FP32 MFMA) for an even nrhs; fmm_tucker_tune may choose differently for an nrhs
 * (it offers both paths at any nrhs for these two precisions).  FMM_C128 takes
 * the matrix cores at every nrhs when the layout's largest item does not fit the FP64
 * streaming kernels' LDS (they keep an item's x_g or core-stage vector and its r_beta
 * or angular intermediate there: about 10,000 complex128 values on 160 KB).  The
 * matrix-core path computes every contraction of
 * Section II.C as one grouped complex GEMM over all (group, polarisation) items for a
 * chunk of right-hand sides (factors read once per chunk); it keeps library-owned
 * device tables and scratch per nrhs (freed by a new
 * upload, fmm_tucker_set_group or fmm_tucker_destroy).  Calls of one handle and
 * precision that use the matrix-core path share that scratch: they must not run
 * concurrently on different streams.  In layouts of fewer than 128 (group,
 * polarisation) items the streaming kernels split large items into blocks of their
 * r_beta rows on several workgroups and sum the blocks' partial results, in block
 * order, in a finishing kernel (TUCKFMM_SPLIT_ELEMS, read at upload, sets the block
 * size in streamed elements for any layout); the partial sums live in a
 * library-owned buffer of the handle, shared the same way. */
typedef enum { FMM_C128 = 0, FMM_C64 = 1, FMM_BF16X2 = 2, FMM_BF16X3 = 3 } fmm_prec;

/* Problem layout shared by every group-wise call. */
typedef struct {
  int32_t n_theta;           /* n_theta = L + 1 angular samples in theta (Section II.A) */
  int32_t n_phi;             /* n_phi samples in phi (2L + 1 in the paper)              */
  int32_t n_groups;          /* number of non-empty boxes                               */
  int32_t reserved;          /* must be 0                                               */
  const int64_t* offsets;    /* host, n_groups + 1 entries, offsets[0] = 0, increasing  */
} fmm_layout;

typedef struct fmm_geometry_s* fmm_geometry_t;   /* mesh, RWG basis, groups, grid   */
typedef struct fmm_tucker_s* fmm_tucker_t;       /* Tucker-compressed far-fields     */
typedef struct fmm_dense_s* fmm_dense_t;         /* plan of the dense (plain) method */

/* ------------------------------------------------------------------ status */

/* Message of the last failing call on this thread ("" if none).  The pointer stays
 * valid until the next library call on the same thread. */
const char* fmm_last_error(void);

/* Library version string, e.g. "tuckfmm 0.2 gfx950 src 0123456789abcdef" (the last
 * word: a hash of the kernel sources the library was built from). */
const char* fmm_version(void);

/* Number of usable HIP devices (0 when no GPU is present).  Never fails. */
int32_t fmm_device_count(void);

/* ---------------------------------------------------------------- geometry */

/* RWG basis functions (Section II.A, the basis of ref. [20]) and FMM groups
 * (Section II.A, the box partition of FMM-FFT) of a triangle mesh, closed or open
 * (e.g. the plates of the trihedral example, Section III.A).  Host only.
 *   verts  host [n_verts][3] double      vertex coordinates (wavelengths)
 *   tris   host [n_tris][3] int32        triangles, counter-clockwise seen from the
 *                                        side the normal points to
 *   origin host [3] double, box > 0, boxes_per_axis >= 1: the cubic box grid;
 *          a basis function belongs to the box holding its edge midpoint,
 *          floor((m - origin) / box) clamped to [0, K-1]; groups are the non-empty
 *          boxes in increasing (ix * K + iy) * K + iz order.
 *   wavenumber k > 0; n_theta >= 1, n_phi >= 1: the angular grid used by
 *          fmm_farfield_fill (Gauss-Legendre nodes in cos(theta), increasing theta;
 *          phi_j = 2 pi j / n_phi).
 * An edge shared by two triangles must be traversed by them in opposite directions
 * and carries one basis function; an edge of one triangle is a free rim and carries
 * none; an edge of three or more triangles, a degenerate edge or a mesh without
 * shared edges is FMM_ERR_SHAPE.  For an edge (a, b), a < b, T+ is the
 * triangle traversing a -> b; basis functions are first ordered by (a, b), then
 * stably by group.  The handle copies everything it needs. */
fmm_status fmm_geometry_build(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                              const double* origin, double box, int32_t boxes_per_axis,
                              double wavenumber, int32_t n_theta, int32_t n_phi,
                              fmm_geometry_t* out);

/* Sizes of a geometry: number of basis functions N and of groups. */
fmm_status fmm_geometry_info(fmm_geometry_t geom, int64_t* n_basis, int32_t* n_groups);

/* Copies of the geometry's tables into caller host buffers (any may be NULL):
 *   offsets [n_groups+1] int64, perm [N] int64 (edge number of each group-ordered
 *   basis function), centers [n_groups][3] double (box centres r_v of eq. (4)),
 *   theta [n_theta] double, phi [n_phi] double. */
fmm_status fmm_geometry_tables(fmm_geometry_t geom, int64_t* offsets, int64_t* perm, double* centers,
                               double* theta, double* phi);

/* A layout view of the geometry (offsets pointer owned by the geometry). */
fmm_status fmm_geometry_layout(fmm_geometry_t geom, fmm_layout* out);

/* The box grid of the FMM-FFT partition (Section II.A): *boxes_per_axis = K (the grid
 * is K x K x K) and box_of_group host int64 [n_groups] = the linear index
 * (ix * K + iy) * K + iz of each group's box (either pointer may be NULL).  These are
 * the arguments fmm_tucker_set_box_grid takes. */
fmm_status fmm_geometry_boxes(fmm_geometry_t geom, int32_t* boxes_per_axis, int64_t* box_of_group);

/* Dense far-fields P^{alpha,+} of eq. (4) for groups first_group ..
 * first_group+count-1, on the device, FP64:
 *   farfield device complex128 [rows][2][n_theta][n_phi], rows = the groups' basis
 *   functions, starting at row offsets[first_group].
 * Each triangle integral uses the symmetric 3-point rule (barycentric
 * (2/3, 1/6, 1/6), weights A/3); the projector (I - k k) drops out because
 * alpha_hat is orthogonal to k.  Uploads the geometry to the device on first use. */
fmm_status fmm_farfield_fill(fmm_geometry_t geom, int32_t first_group, int32_t count,
                             void* farfield, void* stream);

/* Excitation vectors of plane waves, the right-hand side V of eq. (2) (Section II.A):
 * for incident fields E^i(r) = e_hat_r exp(-j k k_hat_r . r) (unit amplitude, phase
 * reference at the origin), Galerkin testing with the RWG functions gives
 *     x[n][r] = < b_n, n x n x E^i_r > = - int_{S_n} b_n(r) . e_hat_r exp(-j k k_hat_r . r) dr
 * (b_n is tangential, so n x n x E reduces to -E there).  Each triangle uses the same
 * symmetric 3-point rule as fmm_farfield_fill; the result is the aggregation input
 * x of eq. (3) for nrhs incident waves at once.
 *   khat   host double [nrhs][3]  unit propagation directions (|k_hat| within 1e-6
 *                                 of 1, else FMM_ERR_ARG)
 *   epol   host double [nrhs][3]  polarisations (orthogonal to k_hat for a physical
 *                                 wave; used as given)
 *   prec   FMM_C128: x is complex128; any other precision: complex64 (each part of
 *          the FP64 sum rounded to the nearest float)
 *   x      device [N][nrhs], basis functions in group order, naturally aligned.
 * FP64 arithmetic.  Uploads the geometry to the device on first use and keeps a
 * small device table of the waves; synchronises the stream before reusing it, then
 * runs asynchronously.  FMM_ERR_NUMERIC for a non-finite direction or polarisation. */
fmm_status fmm_planewave_excitation(fmm_geometry_t geom, int32_t nrhs, const double* khat, const double* epol,
                                    fmm_prec prec, void* x, void* stream);

void fmm_geometry_destroy(fmm_geometry_t geom);

/* ------------------------------------------------------------------ Tucker */

/* Empty Tucker handle for a layout (host only).  Groups are filled by
 * fmm_farfield_compress or fmm_tucker_set_group. */
fmm_status fmm_tucker_create(const fmm_layout* layout, fmm_tucker_t* out);

/* Setup: truncated HOSVD (Section II.B, eq. (6)) of the dense far-fields of groups
 * first_group .. first_group+count-1, one decomposition per group and polarisation.
 *   farfield device complex128 [rows][2][n_theta][n_phi], starting at row
 *            offsets[first_group] (so a caller can stream group chunks).
 *   gamma    tolerance, 0 <= gamma < 1.  Each mode keeps the smallest rank r with
 *            sqrt(sum_{i>=r} s_i^2) <= gamma/sqrt(3) * ||A||_F (gamma = 0: full rank),
 *            so that ||A - A_hat||_F <= gamma ||A||_F.
 * FP64 throughout: the left singular vectors of each mode unfolding come from the
 * Hermitian eigendecomposition of the unfolding's Gram matrix (s_i^2 = eigenvalues),
 * the core is A x_1 U^theta* x_2 U^phi* x_3 U^beta*.  If *inout is NULL a handle is
 * created for the layout, else groups are added to it.  Synchronises the stream. */
fmm_status fmm_farfield_compress(const fmm_layout* layout, const void* farfield, int32_t first_group,
                                 int32_t count, double gamma, void* stream, fmm_tucker_t* inout);

/* Setup of the paper's comparison method, the truncated SVD (Section I; Section II.C,
 * last paragraph): only the basis mode is compressed.  Per (group, polarisation),
 * U^beta (n_beta x r_beta) holds the leading left singular vectors of the basis-mode
 * unfolding, with the smallest r_beta such that sqrt(sum_{i>=r} s_i^2) <= gamma ||A||_F,
 * and W = A conj(U^beta) (N_dir x r_beta), so that A ~ W U^beta^T.  The handle stores
 * it as a Tucker tensor with identity angular factors (r_theta = n_theta,
 * r_phi = n_phi, core[i_theta][i_phi][b] = W[i][b]); the compute calls then apply
 * F = W (U^beta^T x) and V = conj(U^beta) (W^H G) with no angular products, and the
 * storage measure counts U^beta and W only.  Arguments, streaming by group ranges and
 * errors as fmm_farfield_compress; FP64 throughout.  fmm_tucker_set_group with exact
 * identity angular factors gives the same representation. */
fmm_status fmm_farfield_compress_svd(const fmm_layout* layout, const void* farfield, int32_t first_group,
                                     int32_t count, double gamma, void* stream, fmm_tucker_t* inout);

/* Set the factors of one (group, polarisation) from host complex128 arrays in the
 * paper's shapes (see the conventions above).  1 <= r_theta <= n_theta,
 * 1 <= r_phi <= n_phi, 1 <= r_beta <= n_beta.  Copies the data. */
fmm_status fmm_tucker_set_group(fmm_tucker_t h, int32_t group, int32_t alpha, int32_t r_theta,
                                int32_t r_phi, int32_t r_beta, const double* core, const double* u_theta,
                                const double* u_phi, const double* u_beta);

/* Box-grid layout of the spectra (eq. (3) and (5), Section II.A): the outgoing
 * spectra F^alpha_u of eq. (3) are tensors of K_x x K_y x K_z x N_dir entries per
 * polarisation, zero on empty boxes, and the incoming spectra G^alpha_u of eq. (5) are
 * read from the same positions.  After this call every aggregation, disaggregation,
 * pass and graph capture of the handle takes
 *   F, G device [2][K_x][K_y][K_z][N_dir][nrhs]   (alpha, then the box's linear index
 *                                                  (v_x K_y + v_y) K_z + v_z)
 * instead of [n_groups][2][N_dir][nrhs].  Group g's fibre F^alpha_g sits at box
 * box_of_group[g] (host int64 [n_groups], distinct values in [0, K_x K_y K_z)).  The
 * aggregation writes every entry of F: the fibres of the groups, and zero on the
 * empty boxes (an extra fill of (K - n_groups) 2 N_dir nrhs values).  The
 * disaggregation reads only the groups' boxes; entries of G at empty boxes are never
 * read.  kx = ky = kz = 0 with box_of_group = NULL returns to the group-compact layout.
 * Errors: FMM_ERR_ARG (sizes < 1, a box out of range or holding two groups),
 * FMM_ERR_SHAPE (fewer boxes than groups), FMM_ERR_SIZE (more than 2^30 boxes).  Like
 * fmm_tucker_set_group it makes earlier uploads stale: upload again before computing. */
fmm_status fmm_tucker_set_box_grid(fmm_tucker_t h, int32_t kx, int32_t ky, int32_t kz, const int64_t* box_of_group);

/* Save the handle's FP64 factors, ranks, layout and box grid to a binary file (host
 * only), so that the setup of eq. (4) and Section II.B is done once.  Little-endian
 * 8-byte words: magic, version, layout, box grid, then per (group, alpha) the ranks,
 * the identity flag and the four complex128 arrays in fmm_tucker_set_group's shapes,
 * then a checksum (sum of all words mod 2^64).  FMM_ERR_STATE if a tensor is unset,
 * FMM_ERR_IO if the file cannot be written.  Uploads are not saved. */
fmm_status fmm_tucker_save(fmm_tucker_t h, const char* path);

/* Load a handle written by fmm_tucker_save into a new handle (*out; NULL on error).
 * The factors are bit-identical to the saved ones; precisions must be uploaded
 * again.  FMM_ERR_IO for a missing, truncated or corrupt file (checksum, ranks, sizes
 * or identity flags inconsistent). */
fmm_status fmm_tucker_load(const char* path, fmm_tucker_t* out);

/* The handle's layout (offsets pointer owned by the handle, valid until it is
 * destroyed), e.g. to size buffers for a loaded handle. */
fmm_status fmm_tucker_layout(fmm_tucker_t h, fmm_layout* out);

/* Ranks of every tensor: host int32 [n_groups][2][3] = (r_theta, r_phi, r_beta). */
fmm_status fmm_tucker_ranks(fmm_tucker_t h, int32_t* ranks);

/* Copy the factors of one (group, polarisation) of eq. (6) into host complex128
 * buffers in the paper's shapes (sizes from fmm_tucker_ranks; any pointer may be NULL).
 *   as_stored  FMM_C128: the handle's FP64 factors as they are.
 *              FMM_C64, FMM_BF16X2, FMM_BF16X3: every real and imaginary part rounded
 *              to the nearest float and widened back, i.e. exactly the complex64
 *              values an upload of that precision stores (the bf16 pieces of the split
 *              precisions are formed from these on chip).
 * With as_stored = the upload's precision, a plain FP64 contraction of the exported
 * factors (Fig. 2(b), Fig. 3(b)) is the exact result the compute calls approximate:
 * their difference is the arithmetic error alone, free of the compression error.
 * FMM_ERR_ARG for a bad group, alpha or precision; FMM_ERR_STATE if unset. */
fmm_status fmm_tucker_export(fmm_tucker_t h, int32_t group, int32_t alpha, fmm_prec as_stored, double* core,
                             double* u_theta, double* u_phi, double* u_beta);

/* Bytes of stored factors (paper's memory measure, Section III: core + 3 factors of
 * every tensor at the precision's element size), and bytes of the device arena the
 * library needs for that precision (factors with row padding + descriptor tables). */
fmm_status fmm_tucker_storage_bytes(fmm_tucker_t h, fmm_prec prec, size_t* factor_bytes, size_t* arena_bytes);

/* Convert the FP64 factors to `prec` and copy them into the caller's device arena
 * (at least arena_bytes from fmm_tucker_storage_bytes, 256-byte aligned).  The
 * arena must stay allocated and unmodified while the precision is in use; a second
 * upload of the same precision replaces the first.  Synchronises the stream. */
fmm_status fmm_tucker_upload(fmm_tucker_t h, fmm_prec prec, void* arena, size_t bytes, void* stream);

/* Aggregation in Tucker format (Section II.C, Fig. 2(b)) for every group and both
 * polarisations: F^alpha_g = A_hat^alpha_g x_g, A_hat the Tucker model of eq. (6).
 *   x device [N][nrhs], F device [n_groups][2][N_dir][nrhs] (on a box grid:
 *   [2][K_x][K_y][K_z][N_dir][nrhs], see fmm_tucker_set_box_grid); complex128 for
 *   FMM_C128, complex64 otherwise.  Requires a prior upload of `prec`. */
fmm_status fmm_tucker_aggregate(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                void* stream);

/* Disaggregation in Tucker format (Section II.C, Fig. 3(b)), summed over the two
 * polarisations as in eq. (5): V_g = sum_alpha (A_hat^alpha_g)* G^alpha_g, with *
 * the conjugate transpose.  G device [n_groups][2][N_dir][nrhs] (on a box grid:
 * [2][K_x][K_y][K_z][N_dir][nrhs]), V device [N][nrhs]. */
fmm_status fmm_tucker_disaggregate(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* G, void* V,
                                   void* stream);

/* One aggregation + disaggregation pass: F = aggregation of x and V = disaggregation
 * of G exactly as fmm_tucker_aggregate and fmm_tucker_disaggregate compute them (same
 * arithmetic, bitwise equal results), with the work of both stages interleaved in
 * longest-first work lists (streaming kernels: one persistent launch that takes the
 * list's entries from a work counter; matrix-core path: four grouped launches per chunk
 * of right-hand sides).  F must not alias G, x or V.  Passes of one handle and
 * precision must not overlap in time (on different streams): they share the work
 * counter, the partial sums and the multi-RHS scratch. */
fmm_status fmm_tucker_pass(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F, const void* G,
                           void* V, void* stream);

/* Capture fmm_tucker_pass with these buffers into a HIP graph owned by the handle,
 * replacing a previous capture (device tables are built before the capture starts).
 * Buffers must stay valid while the graph is used.  A new upload, set_group or tune
 * call drops the graph (fmm_graph_launch then returns FMM_ERR_STATE). */
fmm_status fmm_graph_capture(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                             const void* G, void* V, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): fmm_tucker_pass with the same
 * arguments, results and errors, computed by the streaming kernels (whatever the
 * route of fmm_tucker_pass for this nrhs) with the pass kernel's work counter (first
 * 256 bytes) and the partial sums of split items in a static device array of 64 MiB
 * per GPU instead of library allocations.  It calls no hipMalloc, hipFree or
 * allocating library routine.
 *   prec  FMM_C128 or FMM_C64 (the bf16 split precisions run only on the matrix-core
 *         path, whose tables the library allocates: FMM_ERR_UNSUPPORTED; so is a layout
 *         whose FP64 items exceed the streaming kernels' LDS).
 * FMM_ERR_SIZE when the split items' partial sums (their r_theta r_phi and n_beta
 * values per block, per right-hand side) exceed the array after the counter: fewer
 * right-hand sides per call, or no split items, fit.  Every call on one GPU shares
 * that GPU's array, which keeps the last call's contents (the kernels overwrite every
 * block they read, and the counter is reset before each pass): calls that overlap on
 * one GPU, from two streams or two threads, race. */
fmm_status fmm_tucker_pass_noalloc(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                   const void* G, void* V, void* stream);

/* Launch the captured pass on `stream`. */
fmm_status fmm_graph_launch(fmm_tucker_t h, void* stream);

/* A kernel configuration for one nrhs: path 0 = streaming kernels with `threads` (64,
 * 128, 256 or 512) per workgroup; path 1 = matrix-core products with `tile_steps` K
 * steps per workgroup, `rhs_chunk` right-hand sides per chunk and the angular
 * contraction `order` (0: each item's cheaper order, 1: U^theta first, 2: U^phi first,
 * for every item); ms = mean time of one pass; from_cache = 1 when fmm_tucker_tune
 * took the result from its cache file. */
typedef struct {
  int32_t path;
  int32_t tile_steps;
  int32_t rhs_chunk;
  int32_t threads;
  float ms;
  int32_t order;
  int32_t from_cache;
} fmm_tune_result;

/* Autotuner: times fmm_tucker_pass with these buffers under each candidate
 * configuration for (prec, nrhs) (1 warm-up + 3 timed passes each, HIP events on the
 * stream): the four streaming workgroup sizes, and on the matrix cores 8, 16, 32 and 64 K
 * steps per tile, up to three chunk sizes and the three angular orders.  Keeps the
 * fastest for later calls with this nrhs and reports it in *out (may be NULL).  With
 * the environment variable TUCKFMM_TUNE_CACHE naming a file, a result stored there
 * for the same layout shapes (groups, ranks, box grid), precision, nrhs and kernel
 * sources is applied without timing (F and V are then left untouched), and a new
 * result is appended to the file.  Otherwise overwrites F and V.  Synchronises the
 * stream; drops a captured graph.  Not allowed while the stream is capturing. */
fmm_status fmm_tucker_tune(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F, const void* G,
                           void* V, void* stream, fmm_tune_result* out);

/* Use `choice` (path, tile_steps, rhs_chunk, threads, order; ms and from_cache are
 * ignored) for later calls of precision `prec` with this nrhs, e.g. a result kept from
 * an earlier fmm_tucker_tune.  FMM_ERR_ARG for values out of range, FMM_ERR_UNSUPPORTED
 * for a path the precision or layout cannot take, FMM_ERR_STATE before an upload.
 * Drops a captured graph; a new upload or set_group forgets the choice. */
fmm_status fmm_tucker_set_tuned(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const fmm_tune_result* choice);

void fmm_tucker_destroy(fmm_tucker_t h);

/* ------------------------------------------------------------------- dense */

/* Plan of the plain method for a layout: uploads the group table and the row-block
 * table of the multi-RHS disaggregation to the current device.  Both stages read each
 * far-field element once per 8 right-hand sides. */
fmm_status fmm_dense_create(const fmm_layout* layout, fmm_dense_t* out);

/* Dense aggregation, eq. (3) / Fig. 2(a): F^alpha_g = A^alpha_g x_g.
 *   farfield device [N][2][n_theta][n_phi] (complex128 for FMM_C128, complex64 for
 *   FMM_C64; other precisions: FMM_ERR_UNSUPPORTED), x [N][nrhs], F as above. */
fmm_status fmm_dense_aggregate(fmm_dense_t d, fmm_prec prec, const void* farfield, int32_t nrhs,
                               const void* x, void* F, void* stream);

/* Dense disaggregation, eq. (5) / Fig. 3(a): V_g = sum_alpha (A^alpha_g)* G^alpha_g. */
fmm_status fmm_dense_disaggregate(fmm_dense_t d, fmm_prec prec, const void* farfield, int32_t nrhs,
                                  const void* G, void* V, void* stream);

void fmm_dense_destroy(fmm_dense_t d);

#ifdef __cplusplus
}
#endif
#endif /* TUCKFMM_H */
