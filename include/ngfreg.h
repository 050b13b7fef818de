/*
 * ngfreg.h - C ABI of the MI355X (gfx950) library for matrix-free NGF +
 * curvature deformable 3D image registration.
 *
 * Method: Budelmann, Koenig, Papenberg, Lellmann, "Fully-deformable 3D image
 * registration in two seconds" (BVM 2019).  The objective is
 *     J(y) = D(R, T(P y)) + alpha S(y)                         (Sec. 2.1, Eq. 1)
 * with D the normalised gradient field distance (Sec. 2.2, Eq. 2), S the
 * curvature regulariser (Sec. 2.1), P the trilinear conversion from the
 * deformation grid to the image grid and P^T its conflict-free gather adjoint
 * (Sec. 2.2, "Grid conversion", Eq. 3).  It is minimised by L-BFGS in a
 * coarse-to-fine scheme (Sec. 2.1) over a multi-level image pyramid
 * (Sec. 2.2, "Generating the multi-level pyramid").
 *
 * Conventions shared by every call
 * --------------------------------
 * Layout.  Images are float32 arrays [m_x][m_y][m_z], z fastest (C order).
 *   A deformation y (and a gradient with respect to y) is float32
 *   [3][m^y_x][m^y_y][m^y_z]: component-major, then x, y, z, z fastest.
 * Grids.  The image grid is cell-centred: voxel i has its centre at
 *   (i + 1/2) h.  The deformation grid is nodal over the same domain
 *   [0, m h]: node j sits at j h^y with h^y = m h / (m^y - 1), and
 *   m^y = m / ratio + 1 per axis at every level.  y holds positions (a
 *   transformation); the identity is y = node positions (ngf_identity).
 * Levels.  Level 0 is the input resolution; level l has m / 2^l cells of
 *   spacing h 2^l per axis; level (levels - 1) is the coarsest.
 * Pointers.  Unless a call says otherwise, every pointer argument is device
 *   memory owned by the caller (for instance a torch tensor), valid for the
 *   duration of the call; the library never frees or retains it.  Work is
 *   enqueued on the context's HIP stream in order; a call returns after its
 *   work is enqueued unless it documents a synchronisation.
 * Ownership.  The context owns every internal buffer (pyramid, index maps,
 *   partial sums, L-BFGS history).  All of them are allocated by
 *   ngf_create / ngf_build_pyramid; the evaluation and L-BFGS calls do not
 *   allocate (ngf_eval_pair may, on its first call for a larger grid).
 * Errors.  No call throws or aborts across the ABI.  Every call returns an
 *   ngf_status; on failure ngf_last_error() describes the cause and the
 *   outputs are left unspecified.  One context per host thread.
 *
 * The method's operations and the calls that carry them
 * ----------------------------------------------------
 *   register(R, T, alpha, levels) -> y   (Sec. 2.1: coarse-to-fine L-BFGS)
 *       ngf_create(params, stream, &ctx) with params.alpha and params.levels,
 *       then ngf_register(ctx, R, T, grid, y, host_ptrs, report).  alpha and
 *       the level count are context parameters (ngf_create, ngf_set_params)
 *       rather than per-call arguments because the pyramid, the index maps,
 *       the partial-sum buffers and the L-BFGS history are sized from them
 *       once, so that no evaluation or iteration allocates.
 *   build_pyramid(R, T)                  (Sec. 2.2)  ngf_build_pyramid
 *   eval_J_grad(level, y) -> J, grad     (Eq. 1-3)   ngf_eval_J_grad
 *   eval_J_grad_T(level, y) -> J, grad_y, grad_T     ngf_eval_J_grad_T
 *   lbfgs_step(level, y) -> y, grad, J   (Sec. 2.1)  ngf_lbfgs_reset(level,
 *       y0) once, then ngf_lbfgs_step per iteration and ngf_lbfgs_get for the
 *       iterate: the iterate, its gradient and the history stay in the
 *       context between steps instead of crossing the ABI every iteration.
 *   prolongate(level, y_c) -> y_f        (Sec. 2.1)  ngf_prolongate
 *   the same over many pairs             ngf_batch_create, ngf_batch_register,
 *       ngf_batch_build + ngf_batch_eval.
 */
#ifndef NGFREG_H
#define NGFREG_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ngf_ctx ngf_ctx;

/* Image grid: cells per axis and spacing per axis (index 0 = x ... 2 = z). */
typedef struct {
    int32_t m[3];
    double h[3];
} ngf_grid;

/* Model and solver parameters.
 *   alpha      regulariser weight (Eq. 1), >= 0
 *   tau, rho   edge parameters of the template and reference gradients (Eq. 2), > 0
 *   levels     pyramid levels, 1..12
 *   ratio      image cells per deformation cell per axis (2: m^y = m/2 + 1)
 *   max_iter   L-BFGS iterations per level, >= 0
 *   lbfgs_mem  stored correction pairs, 1..8
 *   tol_J      relative decrease for the early stop
 *   early_stop 1: stop a level when J falls by at most tol_J (1 + |J|)
 */
typedef struct {
    double alpha;
    double tau;
    double rho;
    int32_t levels;
    int32_t ratio;
    int32_t max_iter;
    int32_t lbfgs_mem;
    double tol_J;
    int32_t early_stop;
    int32_t reserved;
} ngf_params;

typedef enum {
    NGF_OK = 0,
    NGF_E_ARG = -1,       /* null pointer or parameter out of range */
    NGF_E_SHAPE = -2,     /* grid not divisible / too small for the levels */
    NGF_E_STATE = -3,     /* call out of order (e.g. no pyramid built) */
    NGF_E_LEVEL = -4,     /* level index out of range */
    NGF_E_OOM = -5,       /* device allocation failed */
    NGF_E_HIP = -6,       /* a HIP runtime call failed */
    NGF_E_NONFINITE = -7  /* NaN or infinity in an input or in J */
} ngf_status;

/* Outcome of one L-BFGS iteration. */
enum {
    NGF_INFO_OK = 0,              /* step accepted */
    NGF_INFO_CONVERGED = 1,       /* zero gradient or early-stop criterion met */
    NGF_INFO_MAX_ITER = 2,        /* level ended after max_iter iterations */
    NGF_INFO_LINESEARCH_FAIL = 3, /* no Armijo step within 10 halvings; y kept */
    NGF_INFO_NONFINITE = 4        /* J or the gradient is not finite */
};

#define NGF_MAX_LEVELS 12

/* Per-level outcome of ngf_register (index = level). */
typedef struct {
    int32_t levels;
    int32_t iters[NGF_MAX_LEVELS];
    int32_t evals[NGF_MAX_LEVELS];
    int32_t info[NGF_MAX_LEVELS];
    double J[NGF_MAX_LEVELS];
    double ms[NGF_MAX_LEVELS]; /* host wall time of the level: start of the
                                  level to its last queued work done */
} ngf_report;

/* Library version string (static storage). */
const char* ngf_version(void);

/* Create a context.  `stream` is a hipStream_t (NULL = the null stream) on
 * which all work of this context is enqueued.  Errors: NGF_E_ARG for a null
 * `out` / `p` or parameters out of the documented ranges; NGF_E_HIP. */
ngf_status ngf_create(const ngf_params* p, void* stream, ngf_ctx** out);

/* Destroy a context and free everything it owns; NULL is ignored.
 * Synchronises the context's stream first. */
void ngf_destroy(ngf_ctx* ctx);

/* Message of the last failure on this context (static until the next call). */
const char* ngf_last_error(const ngf_ctx* ctx);

/* Replace alpha, tau, rho (and the solver fields) of a context. */
ngf_status ngf_set_params(ngf_ctx* ctx, const ngf_params* p);

/* Build the multi-level pyramid of R and T (Sec. 2.2, "Generating the
 * multi-level pyramid"): level l+1 is the 2x2x2 box mean of level l, summed in
 * float64 in a fixed order and rounded once to float32, bit-identical for
 * identical inputs.  Also builds the per-axis index maps of every level
 * (Sec. 2.2, "Grid conversion": the index sets and weights are determined
 * beforehand per dimension) and sizes all scratch buffers.  The two images
 * are processed on two internal streams that join the context's stream.
 *   R, T       input images on `g` ([m_x][m_y][m_z] float32)
 *   host_ptrs  0: R and T are device pointers; 1: host pointers (copied
 *              host-to-device on the two streams)
 * Shape rule: every m_d divisible by ratio * 2^(levels-1), the coarsest
 * level at least 4 cells and 2 deformation cells per axis, and fewer than
 * 2^30 voxels (32-bit byte offsets into the images); otherwise NGF_E_SHAPE.
 * Synchronises before returning. */
ngf_status ngf_build_pyramid(ngf_ctx* ctx, const float* R, const float* T,
                             const ngf_grid* g, int32_t host_ptrs);

/* Deformation grid of level 0 per axis (Sec. 2.2, "Grid conversion": the
 * index sets and weights of P are fixed per dimension by the two grids, so
 * each axis may have its own node count).  my0[d] = 0 keeps the default
 * m_d / ratio + 1; a NULL my0 resets all three.  Level l then has
 * (my0[d] - 1) / 2^l + 1 nodes along axis d, so ngf_build_pyramid requires
 * my0[d] - 1 divisible by 2^(levels-1), at least 2 node cells on the
 * coarsest level, and between two and sixteen image cells per node cell
 * (2 (my0[d] - 1) <= m_d <= 16 (my0[d] - 1); the ratio need not be an
 * integer), else NGF_E_SHAPE there.  Levels whose
 * grids are m/2 + 1 or m/4 + 1 on every axis may use every image-pass
 * variant; any other grid uses variant 14.  Clears a built pyramid.
 * Errors: NGF_E_ARG for a count in 1..2. */
ngf_status ngf_set_node_grid(ngf_ctx* ctx, const int32_t my0[3]);

/* Image-grid kernel of the evaluation.  `variant`: -2 = by level size (no
 * timing runs: at least 1 Mi voxels -> 13, else 8);
 * -1 = autotune (default:
 * at ngf_build_pyramid every level times each variant over three evaluations
 * at the identity and keeps the fastest; choices are cached per image shape
 * in the context and, if the environment variable NGF_TUNE_CACHE names a
 * file, appended to and read from that file); 0 = 3D tiles of 8x8x32 voxels
 * with a two-voxel halo; 1, 2, 3 = x-marching over 16x64 (y, z) tiles in
 * chunks of 8, 20 or 32 planes; 4, 5, 6 = the same over 16x32 tiles; 7 = 3D
 * tiles of 4x8x32 voxels; 8 = 3D tiles of 4x4x16 voxels; 9, 10 = x-marching
 * over 16x64 or 16x32 tiles in chunks of 16 planes; 11, 12 = x-marching over
 * 16x32 or 16x64 tiles in chunks whose length is fitted to the level's shape
 * and to the number of workgroups the device holds at once (so that the
 * launch fills the device in as few full rounds as possible); 13 = the same
 * over 32x32 tiles with 512-thread workgroups; 14 = x-marching over 32x32
 * tiles reading the exact index maps (any deformation grid, one barrier per
 * plane step, the reference side of the NGF term prepared per pyramid).
 * A variant that needs a ratio of 2 or 4 is replaced by 14 on other grids.
 * All variants
 * compute the same quantities; only the summation order of the P^T partial
 * sums differs.  Applies at once to a built pyramid.  ngf_get_kernel reports
 * a level's choice. */
ngf_status ngf_set_kernel(ngf_ctx* ctx, int32_t variant);
ngf_status ngf_get_kernel(const ngf_ctx* ctx, int32_t level, int32_t* variant);

/* Number of pyramid levels and the grids of one level: `img` gets the image
 * grid, `def` the deformation grid (m = node counts, h = node spacing).
 * Either output may be NULL. */
ngf_status ngf_level_info(const ngf_ctx* ctx, int32_t level, ngf_grid* img, ngf_grid* def);

/* Copy the pyramid images of a level into caller buffers (device, float32,
 * the level's image shape).  Either output may be NULL. */
ngf_status ngf_level_images(ngf_ctx* ctx, int32_t level, float* R_out, float* T_out);

/* Copy one axis of a level's index map into caller device buffers of the
 * level's m_axis entries: j0 (int32 node index), w0, w1 (float32 weights,
 * rounded to nearest from the exact rationals).  Image point i is
 * interpolated from nodes j0[i] (weight w0[i]) and j0[i]+1 (weight w1[i]). */
ngf_status ngf_index_map(ngf_ctx* ctx, int32_t level, int32_t axis,
                         int32_t* j0, float* w0, float* w1);

/* Write the identity deformation (node positions) of a level into y. */
ngf_status ngf_identity(ngf_ctx* ctx, int32_t level, float* y);

/* Objective and gradient at y on a level (Sec. 2.2, "Evaluating the objective
 * function": P, then D with its gradient, then P^T; plus alpha S):
 *   y      deformation of the level (input)
 *   J      host double, receives J(y) (the call synchronises to return it);
 *          may be NULL, then nothing synchronises
 *   grad   device float32, receives grad J(y) (same layout as y); may be NULL
 *   DS     host double[2], receives (D, S); may be NULL
 * J is also kept on the device (see ngf_eval_J_device).  Reductions are
 * float64 with a fixed order, so equal inputs give equal outputs. */
ngf_status ngf_eval_J_grad(ngf_ctx* ctx, int32_t level, const float* y, double* J,
                           float* grad, double* DS);

/* Device address of the double[3] {J, D, S} written by the last evaluation. */
ngf_status ngf_eval_J_device(ngf_ctx* ctx, const double** JDS);

/* The same objective and gradient as ngf_eval_J_grad (Eq. 1-3, Sec. 2.2)
 * with every value in float64, for studies of the float32 arithmetic the
 * paper uses (Sec. 3 compares float32 GPU results with float64 CPU ones):
 * exact rational grid-conversion weights, float64 warp, NGF terms, adjoint,
 * P^T and curvature; the level's float32 images are widened exactly.
 *   y      device float64 [3][m^y_x][m^y_y][m^y_z], the deformation
 *   J      host double, receives J(y); may be NULL (then nothing synchronises)
 *   grad   device float64 like y, receives grad J(y); may be NULL
 *   DS     host double[2], receives (D, S); may be NULL
 * Plain unfused kernels (about 56 bytes of float64 scratch per voxel); the
 * scratch is allocated on the first call and grown when a later call needs a
 * larger level, so this call is not for graph capture.  Reductions have a
 * fixed order: equal inputs give equal outputs.  Not affected by
 * ngf_set_kernel. */
ngf_status ngf_eval_J_grad_f64(ngf_ctx* ctx, int32_t level, const double* y, double* J,
                               double* grad, double* DS);

/* Start L-BFGS (Sec. 2.1; Nocedal 1980) on a level from y0 (device): drops the
 * stored pairs and evaluates J and grad J at y0.  Synchronises. */
ngf_status ngf_lbfgs_reset(ngf_ctx* ctx, int32_t level, const float* y0);

/* One L-BFGS iteration on the level given to ngf_lbfgs_reset: direction by
 * the two-loop recursion (float64 inner products), Armijo backtracking
 * (c1 = 1e-4, halving, at most 10 halvings), pair update.  `J` (host, may be
 * NULL) receives the objective after the iteration, `info` (host, may be
 * NULL) one of NGF_INFO_*.  Synchronises once per trial evaluation. */
ngf_status ngf_lbfgs_step(ngf_ctx* ctx, double* J, int32_t* info);

/* Copy the current L-BFGS iterate and its gradient into caller device
 * buffers (either may be NULL); `J` (host, may be NULL) gets J there. */
ngf_status ngf_lbfgs_get(ngf_ctx* ctx, float* y, float* grad, double* J);

/* Checkpoint and resume of an L-BFGS level (Sec. 2.1: the iterate and the
 * stored correction pairs are the whole state of the method between two
 * iterations).  ngf_lbfgs_save writes the state left by ngf_lbfgs_reset and
 * ngf_lbfgs_step calls into a host buffer: the level, its deformation-grid
 * shape, the iterate y and its gradient, J and the evaluation count, the
 * device state block (Gram matrix of the stored pairs and the gradient, ring
 * order, control block) and the stored pairs (s, t) of the slots in use.
 * ngf_lbfgs_load puts such a state back, into this context or another one
 * of the same library build with a pyramid of the same shapes and the same
 * L-BFGS memory; the ngf_lbfgs_step calls that follow take the same steps,
 * bit for bit, as they would have taken after the save.
 *   ngf_lbfgs_state_size  *bytes: the size of the state as it stands now
 *                         (it depends on the number of stored pairs)
 *   ngf_lbfgs_save        buf: host memory of at least that size; bytes: its
 *                         size.  Synchronises.
 *   ngf_lbfgs_load        buf, bytes: a saved state.  Synchronises.
 * Errors: NGF_E_STATE before ngf_lbfgs_reset (save) or without a pyramid
 * (load); NGF_E_ARG for a null buffer, a buffer too small, or bytes that are
 * not a state of this build (wrong header, size or memory); NGF_E_SHAPE when
 * the saved level's grid differs from this context's level of that index;
 * NGF_E_LEVEL when this context has no such level. */
ngf_status ngf_lbfgs_state_size(const ngf_ctx* ctx, size_t* bytes);
ngf_status ngf_lbfgs_save(ngf_ctx* ctx, void* buf, size_t bytes);
ngf_status ngf_lbfgs_load(ngf_ctx* ctx, const void* buf, size_t bytes);

/* Prolongate a deformation from level `coarse_level` to the next finer level
 * (coarse-to-fine scheme of Sec. 2.1): along each axis fine node 2j takes
 * coarse node j, fine node 2j+1 the mean of coarse nodes j and j+1.  Only for
 * ratio-aligned grids (fine m^y - 1 = 2 (coarse m^y - 1)). */
ngf_status ngf_prolongate(ngf_ctx* ctx, int32_t coarse_level, const float* y_c, float* y_f);

/* Full registration (Sec. 2.1, Sec. 2.2): build the pyramid of R and T, then
 * for each level from the coarsest, start at the identity (coarsest) or the
 * prolongated result, and run L-BFGS until max_iter, a failed line search, a
 * zero gradient or (early_stop) the relative-decrease criterion.
 *   y_out      receives the finest-level deformation ([3][m^y] float32),
 *              device or host memory according to host_ptrs
 *   rep        host, may be NULL: per-level iterations, evaluations, J, info
 * Synchronises before returning. */
ngf_status ngf_register(ngf_ctx* ctx, const float* R, const float* T, const ngf_grid* g,
                        float* y_out, int32_t host_ptrs, ngf_report* rep);

/* Who drives the line search of ngf_register / ngf_register_levels.
 *   mode 0 (default): the device.  Each L-BFGS round (direction or halved
 *     step, trial evaluation, Armijo test, history update, stopping tests) is
 *     a fixed sequence of kernels that read and advance a control block in
 *     device memory; the host enqueues rounds in batches of up to 16 and
 *     reads the control block once per batch.
 *   mode 1: the host, through ngf_lbfgs_step, reading J back after every
 *     trial evaluation.
 * Both take the same decisions on the same numbers: results are identical
 * bit for bit.  Errors: NGF_E_ARG for another mode. */
ngf_status ngf_set_driver(ngf_ctx* ctx, int32_t mode);

/* As ngf_register, from the pyramid already built by ngf_build_pyramid
 * (device-resident inputs; the pyramid step is not repeated). */
ngf_status ngf_register_levels(ngf_ctx* ctx, float* y_out, ngf_report* rep);

/* Differentiation form (for an autograd wrapper): J(y; R, T) on an explicit
 * image pair (not the pyramid) and its gradients with respect to y and to
 * the template T.  The backward is a scatter: each image tile adds its P^T
 * block into grad_y with float atomic additions, and every image point adds
 * e[i] W(i -> k) into grad_T[k] for the 8 corners k of its warp cell (the
 * transpose of the trilinear warp, with e = G^T v the NGF sensitivity of
 * the warped template), so these gradients are reproducible only up to
 * rounding; alpha grad S is added by the node pass.  Sec. 2.1 (Eq. 1),
 * Sec. 2.2 (Eq. 2 and the matrix-free chain rule).
 *   g, my      image grid; my[d] must be m[d]/ratio + 1 (else NGF_E_SHAPE)
 *   R, T, y    device inputs in the usual layouts
 *   gscale     device double multiplying both gradients (the upstream
 *              gradient of an autograd graph), or NULL for 1
 *   J          host double (the call then synchronises) or NULL
 *   J_dev      device double receiving J without synchronising, or NULL
 *   grad_y     device float32 like y, or NULL; grad_T device float32 like T,
 *              or NULL; both NULL: only J is computed, with the plain
 *              evaluation's kernels (no scatter)
 * Allocates index maps and scratch on the first call for a new grid. */
ngf_status ngf_eval_pair(ngf_ctx* ctx, const ngf_grid* g, const int32_t my[3],
                         const float* R, const float* T, const float* y,
                         const double* gscale, double* J, double* J_dev,
                         float* grad_y, float* grad_T);

/* ngf_eval_pair without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * ngf_eval_pair; the pair's index maps and the partial sums live in a static
 * device array of 2 MiB per device (held until the process ends), so the
 * grid is limited to what fits there (about 512^3 voxels; larger grids get
 * NGF_E_SHAPE with the bytes needed).  The ratio is the context's (2 or 4).
 * Every call on one device shares that array and leaves its contents
 * behind: calls that overlap on one device (several contexts or streams at
 * once) race and must be serialised by the caller.  Nothing is cleared with
 * a memset (the partial sums are written before they are read, the
 * gradients are zeroed by a fill kernel), so with J == NULL the call can be
 * captured. */
ngf_status ngf_eval_pair_static(ngf_ctx* ctx, const ngf_grid* g, const int32_t my[3],
                                const float* R, const float* T, const float* y,
                                const double* gscale, double* J, double* J_dev,
                                float* grad_y, float* grad_T);

/* The differentiation form on a pyramid level (Sec. 2.1, Eq. 1; Sec. 2.2,
 * Eq. 2 and the matrix-free chain rule): J at y on level `level` with its
 * gradients with respect to y and to the level's template image, computed
 * as by ngf_eval_pair (atomic scatter of the P^T blocks and of e W(i -> k)
 * into the warp corners) but on the pyramid's images and index maps, with
 * buffers sized by ngf_build_pyramid: nothing is allocated, so the call can
 * be captured in a graph when J is NULL.
 *   y       device float32 deformation of the level
 *   gscale  device double multiplying both gradients, or NULL for 1
 *   J       host double (the call then synchronises) or NULL
 *   J_dev   device double receiving J, or NULL
 *   grad_y  device float32 like y, or NULL
 *   grad_T  device float32 of the level's image shape, or NULL
 * Errors: NGF_E_SHAPE on a level whose deformation grid is not m/2 + 1 or
 * m/4 + 1 on every axis (the scatter kernel holds those ratios);
 * NGF_E_NONFINITE when J is requested and not finite. */
ngf_status ngf_eval_J_grad_T(ngf_ctx* ctx, int32_t level, const float* y, const double* gscale,
                             double* J, double* J_dev, float* grad_y, float* grad_T);

/* Grid conversion as standalone operators on a level's grids (Sec. 2.2,
 * "Grid conversion"; the evaluation fuses them and does not call these).
 *   ngf_apply_P:  yhat = P y, yhat float32 [3][m_x][m_y][m_z] (float64 sums)
 *   ngf_apply_PT: out = P^T z, z like yhat, out like y; `scheme` selects how
 *     the write conflicts of P^T are avoided: 0 = gather, one thread per node
 *     summing its index sets (Eq. 3, the paper's scheme); 1 = scatter with
 *     float atomic additions, one thread per image point (the earlier GPU
 *     scheme the paper cites); 2 = red-black: the slices of the odd x cells
 *     in parallel, then those of the even ones (the earlier scheme the paper
 *     cites); within a cell one thread per (y, z) node sums the cell's slices
 *     over its index sets and adds them to the two node planes of the cell.
 *     Results agree up to the order of float32 sums. */
ngf_status ngf_apply_P(ngf_ctx* ctx, int32_t level, const float* y, float* yhat);
ngf_status ngf_apply_PT(ngf_ctx* ctx, int32_t level, const float* z, float* out,
                        int32_t scheme);

/* Profiling aid: when enabled, the library records HIP events around every
 * launch of the fused image-grid kernel (the dominant kernel of an
 * evaluation) on the context's stream, on pyramid level `level` only (-1:
 * every launch; each record adds two event markers to the stream, a few
 * microseconds of device time).  ngf_kernel_time returns, for the
 * recorded launches on pyramid level `level` (-1: all launches), their
 * number, their summed duration in milliseconds, and the image voxels and
 * deformation nodes they covered; it then clears the whole record and
 * synchronises.  At most 4096 launches are recorded (later ones are not);
 * evaluation rounds enqueued after a device-driven level has ended are not
 * counted.  Any output pointer may be NULL. */
ngf_status ngf_set_profiling(ngf_ctx* ctx, int32_t enable, int32_t level);
ngf_status ngf_kernel_time(ngf_ctx* ctx, int32_t level, int32_t* launches, double* total_ms,
                           int64_t* voxels, int64_t* nodes);

/* Per-iteration record of the L-BFGS levels (the quantities Sec. 2.1 and
 * Sec. 3 speak of, one record per accepted step, plus one for the start
 * point of every level). */
typedef struct {
    int32_t level;   /* pyramid level */
    int32_t iter;    /* accepted steps on the level so far (0: its start point) */
    int32_t evals;   /* J + grad J evaluations on the level so far */
    int32_t reserved;
    double J, D, S;  /* objective (Eq. 1) and its two terms at the iterate */
    double gmax;     /* max |grad J| at the iterate */
    double t;        /* step length of the accepted step (0 at the start) */
    double us;       /* time since the previous record of the level: device
                        clock for the device-driven search, host clock for the
                        host-driven one (0 at the start) */
} ngf_iter_record;

/* Iteration log.  ngf_set_iteration_log(ctx, 1) starts recording (and
 * clears the log), 0 stops.  While on, ngf_lbfgs_reset adds the start record
 * of its level and every accepted step adds one record, in both drivers
 * (ngf_set_driver), which give the same records apart from `us`;
 * ngf_register and ngf_register_levels clear the log first.  The
 * device-driven search then adds one single-lane kernel per round and its
 * records are copied back at the end of each level; its buffer (one record
 * per possible step of a level) is allocated when a level needs a larger one.
 * The batched form records nothing.
 * ngf_iteration_log copies up to `cap` records, oldest first, into `out`
 * (host; may be NULL when cap is 0) and sets *count to the number recorded.
 * Errors: NGF_E_ARG for a negative cap or a null count. */
ngf_status ngf_set_iteration_log(ngf_ctx* ctx, int32_t enable);
ngf_status ngf_iteration_log(const ngf_ctx* ctx, ngf_iter_record* out, int32_t cap,
                             int32_t* count);

/* Failure injection, for tests of the error paths (no other use).  `flags`
 * is a bit set; 0 clears it.
 *   NGF_FAULT_REJECT_STEPS  every L-BFGS trial point fails the Armijo test
 *     (Sec. 2.1, L-BFGS line search), so each iteration ends after its 11
 *     trial evaluations with NGF_INFO_LINESEARCH_FAIL and y unchanged; both
 *     drivers (ngf_set_driver) honour it.  Takes effect at the next
 *     ngf_lbfgs_reset (and so at every level of ngf_register).
 *   NGF_FAULT_ALLOC  every device allocation the context attempts from now
 *     on fails as if the device were out of memory: the call returns
 *     NGF_E_OOM and the context stays usable once the flag is cleared
 *     (buffers already allocated are kept).
 * Errors: NGF_E_ARG for unknown bits. */
#define NGF_FAULT_REJECT_STEPS 1
#define NGF_FAULT_ALLOC 2
ngf_status ngf_set_faults(ngf_ctx* ctx, int32_t flags);

/* Batched form: many independent registrations (one image pair each, any
 * mix of shapes) on one device, each computed as by ngf_register (Sec. 2:
 * pyramid, multi-level L-BFGS on Eq. 1).  Two modes (ngf_batch_set_mode):
 *   0 (default) graph: the pairs go through the levels together; at each
 *     level one L-BFGS round of every pair is one fixed sequence of batched
 *     launches (each covering all pairs through a block table), captured as
 *     a hipGraph and replayed on the batch's own stream until every pair's
 *     level has ended.  Image-pass variants by the timed selection, one
 *     table shared by the pairs (ngf_batch_set_kernel overrides).
 *   1 threads: a host scheduler hands pairs, largest voxel count first, to
 *     `workers` threads (1..16), each with a context on its own stream;
 *     variants by the size rule unless set.
 * In both, every pair's result equals the single-pair ngf_register result
 * for the same image-pass variants bit for bit.
 *   ngf_batch_create      params as for ngf_create; workers as above (used
 *                         by mode 1); the device is the current one
 *   ngf_batch_set_kernel  variant as for ngf_set_kernel, for every pair
 *   ngf_batch_register    npairs >= 0; R[i], T[i]: device float32 images of
 *                         grids[i]; y_out[i]: device float32
 *                         [3][m0/ratio+1][m1/ratio+1][m2/ratio+1]; `stream`
 *                         (hipStream_t, NULL = null stream): the call first
 *                         waits for the work queued there, so the inputs may
 *                         come from it; reports: NULL or npairs entries.
 *                         Synchronous: returns when every pair is done.  On
 *                         failure the status is returned and
 *                         ngf_batch_last_error names the pair; the outputs
 *                         are then unspecified.  Mode 0 keeps one context
 *                         per pair slot between calls (memory grows with
 *                         the largest batch). */
#define NGF_BATCH_MAX_WORKERS 16
typedef struct ngf_batch ngf_batch;
ngf_status ngf_batch_create(const ngf_params* p, int32_t workers, ngf_batch** out);
void ngf_batch_destroy(ngf_batch* b);
const char* ngf_batch_last_error(const ngf_batch* b);
ngf_status ngf_batch_set_kernel(ngf_batch* b, int32_t variant);
ngf_status ngf_batch_set_mode(ngf_batch* b, int32_t mode);
ngf_status ngf_batch_register(ngf_batch* b, int32_t npairs, const float* const* R,
                              const float* const* T, const ngf_grid* grids,
                              float* const* y_out, void* stream, ngf_report* reports);

/* The batched evaluation (Sec. 2.1, Eq. 1 and 2, applied pair by pair):
 * J and grad J of many pairs at given deformations, each stage one launch
 * covering all pairs (one image pass per image-pass variant in use, one node
 * pass, one reduction).  Every pair's J and gradient equal those of the
 * single-pair ngf_eval_J_grad with the same variant bit for bit.
 *   ngf_batch_build  builds the pyramids of npairs pairs (R[i], T[i]: device
 *                    float32 images of grids[i]) in the batch's pair
 *                    contexts (the ones graph mode registers with; an
 *                    ngf_batch_register in graph mode leaves its pairs built
 *                    as well); `stream` as for ngf_batch_register.
 *                    Allocates; synchronises.
 *   ngf_batch_eval   at pyramid level `level` of every built pair: y[i]
 *                    device float32 [3][m^y of that level] (ngf_level_info),
 *                    J (host, npairs doubles, or NULL), grad (NULL for J
 *                    only, else npairs device float32 buffers like y[i]);
 *                    ordered after the work queued on `stream`;
 *                    synchronises.  Allocates only when the batch's table
 *                    buffer or the pinned J buffer must grow.
 * Errors: NGF_E_STATE before any build, NGF_E_LEVEL for a level a pair does
 * not have, NGF_E_ARG for null pointers. */
ngf_status ngf_batch_build(ngf_batch* b, int32_t npairs, const float* const* R,
                           const float* const* T, const ngf_grid* grids, void* stream);
ngf_status ngf_batch_eval(ngf_batch* b, int32_t level, const float* const* y, double* J,
                          float* const* grad, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NGFREG_H */
