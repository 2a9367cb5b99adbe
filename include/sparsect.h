/*
 * sparsect -- precomputed sparse Radon operators for TV-regularised
 * parallel-beam CT on AMD Instinct MI355X (gfx950).
 *
 * The library applies the parallel-beam Radon transform R restricted to the
 * measured angles (the "row selector" M of eq:objmin, Section 1 of Barnard &
 * Archibald, "Accelerating optimization-based computed tomography via sparse
 * matrix approximations") and its adjoint as precomputed sparse matrices, the
 * principle of Section 3 (the geometry is fixed, so the operator is built
 * once, offline, and every evaluation inside the solver becomes a sparse
 * product).  On top of that it provides the normal operator of eq:KKT,
 * eq:PD_resolve and eq:SB_solve (Section 2), conjugate gradients for those
 * systems, and anisotropic-TV split Bregman (Section 4); the Chambolle-Pock
 * method whose primal step is eq:PD_resolve; the surrogate T of Section 3.2;
 * and the Fourier-domain problem of Section 3.1 (eq:four_obj, eq:SBFFT) with
 * its convolution-fused normal operator (eq:fusedop).
 *
 * Geometry (the paper leaves it open; this is the library's convention):
 *   image of n x n unit pixels on [-n/2, n/2]^2, pixel (iy, ix) covers
 *   [ix - n/2, ix - n/2 + 1) x [iy - n/2, iy - n/2 + 1), flat index iy*n + ix;
 *   angles theta_k = pi*k/n_angles, k = 0..n_angles-1; bins
 *   s_b = b - (n_bins - 1)/2; ray (k, b) is the line p.(cos, sin) = s_b.
 *   Entry (ray, pixel) is the length of the ray inside the pixel (Siddon).
 *   A ray exactly on a pixel edge gives half of each length to the two pixels
 *   sharing the edge; lengths <= 1e-12 are dropped.
 *
 * Conventions for every call:
 *   - Device pointers are HIP device memory owned by the caller (the Python
 *     binding passes torch tensors).  The operator's matrix storage is either
 *     caller-owned (radon_csr_sizes, then build_radon_csr_into fills buffers
 *     the caller allocated; the handle borrows them) or allocated by
 *     build_radon_csr and released by radon_op_destroy.
 *   - Compute calls enqueue on `stream` (a hipStream_t; NULL = default
 *     stream) and return without synchronising.  build_radon_csr and the
 *     export calls synchronise.
 *   - Images are laid out [batch][n*n]; measured sinograms [batch][n_meas][n_bins]
 *     with the measured angles in ascending order.  Vector elements are float
 *     for SPARSECT_F32 and double for SPARSECT_F64 and SPARSECT_F32_F64.
 *     SPARSECT_F32_F64 streams the matrix in FP32 (the bandwidth-bound part)
 *     but keeps every vector and every multiply-add in FP64: CG iterates in
 *     FP32 drift from the exact-arithmetic iterates by the conditioning of the
 *     normal operator times the FP32 rounding, which exceeds 1e-5 relative
 *     within ten iterations on the workloads this library targets, while the
 *     FP32 rounding of the matrix entries alone stays near 1e-6.
 *   - Every call returns RADON_OK (0) or a negative status; radon_last_error()
 *     returns a message for the calling thread's most recent failure.
 *   - Argument checks happen before anything is enqueued.
 *   - Results are deterministic: every output element and every partial sum
 *     is written by exactly one thread, and all reductions run in a fixed
 *     order.  No floating-point atomics are used.  The one integer atomic on
 *     an apply path is the work ticket of the mixed-batch forward product
 *     (radon_multi_apply, radon_multi_cg): it only decides which workgroup
 *     takes which ray bundle next, never the order of any sum.
 */
#ifndef SPARSECT_H
#define SPARSECT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPARSECT_F32     0   /* FP32 matrix values, FP32 vectors */
#define SPARSECT_F64     1   /* FP64 matrix values, FP64 vectors */
#define SPARSECT_F32_F64 2   /* FP32 matrix values, FP64 vectors and arithmetic */

#define RADON_OK            0
#define RADON_EINVAL       -1   /* bad argument */
#define RADON_EOVERFLOW    -2   /* a size does not fit the index types */
#define RADON_EHIP         -3   /* a HIP runtime call failed (message has the HIP error) */
#define RADON_EWORKSPACE   -4   /* workspace pointer NULL or too small */
#define RADON_ESTATE       -5   /* operator handle unusable */
#define RADON_EUNSUPPORTED -6   /* valid request the library does not implement */

typedef struct radon_op radon_op;   /* opaque operator handle */

typedef struct {
    int32_t n;                  /* image side, 1 <= n <= 32767 */
    int32_t n_angles;           /* angles theta_k = pi*k/n_angles, >= 1 */
    int32_t n_bins;             /* detector bins, 1 <= n_bins <= 65535 */
    int32_t dtype;              /* SPARSECT_F32, SPARSECT_F64 or SPARSECT_F32_F64 */
    const uint8_t *measured;    /* host array of n_angles flags (nonzero = measured),
                                   NULL = every angle measured; at least one set */
    int32_t fwd_bundle;         /* rays per bundle of the forward layout: 16, 32 or
                                   64 (0 = 16); a layout choice only, the products
                                   equal each other to rounding */
    int32_t fwd_angles;         /* consecutive measured angles per forward bundle:
                                   1, 2 or 4 (0 = 1), with fwd_bundle / fwd_angles
                                   >= 16 adjacent bins of each; a layout choice
                                   only, like fwd_bundle */
    int32_t fwd_compact;        /* 1: the forward layout stores one length per
                                   slot and derives the second (see below); 0:
                                   both stored */
    int32_t fwd_symmetric;      /* 1: the forward layout stores only the measured
                                   angles in [0, pi/4] and serves the rays of
                                   pi - theta, pi/2 - theta and pi/2 + theta from
                                   them (see below), and so does the adjoint
                                   layout when n is a multiple of 8; needs
                                   n >= 2, an even n_angles and a measured set
                                   closed under those maps */
} radon_geom;

typedef struct {
    int64_t n_pixels;           /* n*n */
    int64_t n_meas_angles;      /* measured angles */
    int64_t n_meas_rays;        /* n_meas_angles * n_bins = length of a measured sinogram */
    int64_t nnz;                /* nonzeros of MR (equal to those of (MR)^T) */
    int64_t fwd_slots;          /* slots of the ray-bundle layout (see below) */
    int64_t adj_slots;          /* slots of the pixel-group layout */
    int64_t device_bytes;       /* device memory held by the operator */
    int32_t dtype;
    int32_t n, n_angles, n_bins;
    int32_t needs_transpose;    /* 1: some measured angle is closer to horizontal
                                   than vertical, so the forward product gathers
                                   from the transposed image too */
    int32_t fwd_bundle;         /* rays per forward bundle (16, 32 or 64) */
    int32_t fwd_angles;         /* measured angles per forward bundle (1, 2 or 4) */
    int32_t fwd_compact;        /* 1: compact forward layout */
    int32_t fwd_symmetric;      /* 1: forward layout stored by symmetry */
    int32_t adj_symmetric;      /* 1: adjoint layout stored by symmetry too */
    int32_t reserved;
} radon_info;

/*
 * build_radon_csr -- precompute MR and (MR)^T for one geometry (Section 3:
 * the matrices depend only on the detector, the angle set and the image
 * size, so they are built once, offline).
 *
 * On the GPU it traces every measured ray through the pixel grid (Siddon;
 * FP64 geometry, entries rounded once to the operator dtype) and stores:
 *   - the CSR of MR: row = measured ray (angle-major, bins ascending), entries
 *     in the order the ray visits the pixels (int64 row pointers, int32 pixel
 *     indices);
 *   - a ray-bundle layout of MR for the forward product: groups of
 *     g->fwd_bundle (16, 32 or 64) rays, g->fwd_bundle / g->fwd_angles
 *     adjacent bins of each of g->fwd_angles consecutive measured angles of
 *     one gather class, one slot per (ray, image line along the ray's major
 *     axis) holding the first pixel's offset along that line (uint16) and
 *     the lengths in that pixel and the next one (a ray meets at most two
 *     adjacent pixels of any line along its major axis).  With
 *     g->fwd_compact the second length is not stored: it is the ray's chord
 *     minus the first on every line the ray crosses from side to side (the
 *     two lengths add up to the same chord there), and is kept per ray for
 *     its first and last lines, the only ones it can cross in part.  With
 *     g->fwd_symmetric only the rays of the measured angles in [0, pi/4]
 *     have slots: the rays of pi - theta, pi/2 - theta and pi/2 + theta with
 *     the same bin are their images under x -> -x, the transpose and both,
 *     and the forward reads their lengths from the stored ray's slots;
 *   - a pixel-group layout of (MR)^T for the adjoint: groups of 64 pixels,
 *     one slot per (pixel, measured angle) holding the first bin crossing
 *     the pixel (uint16) and the lengths for that bin and the next one (a
 *     pixel meets at most two adjacent bins of any angle).  With
 *     g->fwd_symmetric and n a multiple of 8 only the angles in [0, pi/4]
 *     have slots: pixel (px, py) meets the rays of pi - theta, pi/2 - theta
 *     and pi/2 + theta as pixel (n-1-px, py), (py, px) and (py, n-1-px)
 *     meets those of theta, bin for bin.
 * Both layouts hold exactly the CSR's values, except that a compact
 * ray-bundle layout's derived second lengths differ from the CSR's by about
 * one rounding of the matrix type relative to the chord (the build checks
 * every line against the chord to 1e-9); the CSR and the adjoint keep the
 * stored values.
 *
 *   g       geometry (host struct); `measured` is read during the call only.
 *   stream  stream for the build kernels; the call synchronises it.
 *   out     receives the handle (host object owning its device storage).
 * Errors: RADON_EINVAL (geometry out of range), RADON_EOVERFLOW (nnz or a
 * layout needs >= 2^31 entries per index type it uses), RADON_EUNSUPPORTED
 * (fwd_angles > 1 and the measured angles fall into more than four runs of
 * one gather class, which angles in index order never do; fwd_symmetric and
 * the measured set is not closed under the maps above, or n_angles is odd;
 * or a layout assumption above failed for some ray), RADON_EHIP.
 */
int build_radon_csr(const radon_geom *g, void *stream, radon_op **out);

/*
 * Caller-owned storage.  radon_csr_sizes counts the entries of every measured
 * ray on the GPU and reports the exact sizes of each array of the operator;
 * the caller allocates them (torch tensors in the Python binding) and
 * build_radon_csr_into fills them.  The library allocates no device memory
 * on this path; the handle it returns borrows the buffers, which must stay
 * allocated and unmodified until radon_op_destroy.  build_radon_csr is the
 * same build with the library allocating (and the handle owning) the arrays.
 */
typedef struct {
    int64_t n_meas_rays;    /* rows of MR */
    int64_t nnz;            /* nonzeros of MR (= of (MR)^T); -1 after a size-only query */
    int64_t fwd_slots;      /* slots of the ray-bundle layout */
    int64_t adj_slots;      /* slots of the pixel-group layout */
    int64_t row_ptr_bytes;  /* int64 row pointers [n_meas_rays + 1] */
    int64_t col_bytes;      /* int32 pixel indices [nnz] */
    int64_t val_bytes;      /* values [nnz] in the matrix type (FP32, or FP64 for SPARSECT_F64) */
    int64_t layout_bytes;   /* one block holding the forward and adjoint layouts and their work orders */
    int64_t ws_bytes;       /* device workspace of radon_csr_sizes and build_radon_csr_into */
} radon_sizes;

typedef struct {
    int64_t *row_ptr;       /* device, >= row_ptr_bytes: receives the CSR row pointers */
    int32_t *col;           /* device, >= col_bytes: receives the CSR pixel indices */
    void *val;              /* device, >= val_bytes: receives the CSR values */
    void *layout;           /* device, >= layout_bytes: receives the derived layouts */
    void *ws;               /* device, >= ws_bytes: scratch during the build only */
    int64_t row_ptr_bytes, col_bytes, val_bytes, layout_bytes, ws_bytes;
} radon_buffers;

/*
 * radon_csr_sizes -- exact storage sizes of the operator of geometry g
 * (Section 3: the sparse operator is built once for the fixed geometry).
 *   ws == NULL: host-only query; fills out->n_meas_rays and out->ws_bytes
 *               (the workspace this call and build_radon_csr_into need),
 *               sets out->nnz = -1, enqueues nothing.
 *   ws != NULL: device workspace of >= ws_bytes (256-byte aligned); runs the
 *               per-ray count kernels on `stream`, synchronises it and fills
 *               every field of *out.
 * Errors: as build_radon_csr; RADON_EWORKSPACE for a short workspace.
 */
int radon_csr_sizes(const radon_geom *g, void *ws, int64_t ws_bytes, void *stream,
                     radon_sizes *out);

/*
 * build_radon_csr_into -- build_radon_csr into caller-allocated buffers (each
 * pointer 256-byte aligned, each size at least the one radon_csr_sizes
 * reported for the same geometry).  The contents are bitwise those
 * build_radon_csr produces.  Synchronises `stream`; the workspace is free
 * for other use once the call returns.
 * Errors: as build_radon_csr; RADON_EINVAL for NULL or misaligned buffers;
 * RADON_EWORKSPACE for a buffer smaller than its array.
 */
int build_radon_csr_into(const radon_geom *g, const radon_buffers *b, void *stream, radon_op **out);

/* Sizes of a built operator (host call, no device work). */
int radon_op_info(const radon_op *op, radon_info *out);

/* Release the operator's device storage and the handle.  NULL is a no-op.
 * The caller must ensure no enqueued work still uses the operator. */
void radon_op_destroy(radon_op *op);

/* Message for the calling thread's most recent failed call ("" if none). */
const char *radon_last_error(void);

/*
 * Layouts of batched vectors (the `layout` argument of radon_fwd, radon_adj,
 * normal_apply, cg_solve and split_bregman_tv):
 *   RADON_LAYOUT_IMAGE  [batch][count]: image (or sinogram) b is contiguous,
 *                       element i of image b at b*count + i;
 *   RADON_LAYOUT_PIXEL  [count][batch]: the batch is interleaved, element i
 *                       of image b at i*batch + b (count = n*n for images,
 *                       n_meas_rays for sinograms).
 * Every input and output of one call uses the call's layout; with batch = 1
 * the two are the same.  The products run image-major; a pixel-major call
 * with batch > 1 relays its inputs and outputs through the end of its
 * workspace (one tiled transpose each way, ordered on the call's stream) and
 * computes exactly what the image-major call computes.
 */
#define RADON_LAYOUT_IMAGE 0
#define RADON_LAYOUT_PIXEL 1

/* Workspace kinds for radon_workspace_bytes. */
#define RADON_WS_FWD      0
#define RADON_WS_NORMAL   1
#define RADON_WS_CG       2
#define RADON_WS_SB       3
#define RADON_WS_PD       4
#define RADON_WS_TUNE     5
#define RADON_WS_ADJ      6
/* OR'ed into RADON_WS_FWD, _ADJ, _NORMAL, _CG or _SB: the size for a
 * pixel-major call (RADON_LAYOUT_PIXEL), which adds its relay buffers after
 * the image-major workspace. */
#define RADON_WS_PIXEL_LAYOUT 0x100

/* Bytes of device workspace a call of the given kind needs for `batch`
 * right-hand sides (>= 0; negative = error status).  The sizes depend on the
 * operator's tuning at the time of the query (radon_set_tuning). */
int64_t radon_workspace_bytes(const radon_op *op, int32_t which, int32_t batch);

/*
 * radon_fwd -- y = M R x for `batch` images (the data term of eq:objmin).
 *   x       device, batch images of n*n, operator dtype, read only.
 *   y       device, batch sinograms of n_meas_rays, written.
 *   layout  RADON_LAYOUT_IMAGE or RADON_LAYOUT_PIXEL (both x and y).
 *   ws      device workspace of radon_workspace_bytes(op, RADON_WS_FWD, batch)
 *           bytes (| RADON_WS_PIXEL_LAYOUT for a pixel-major call).  It holds
 *           the transposed image the ray-bundle layout gathers from for rays
 *           closer to horizontal than vertical and, when the product runs in
 *           line bands (images from 1024 pixels on, and fused chunks whose
 *           images overflow the cache budget), one partial sum per ray and
 *           band, added in band order; with fwd_layout = 1 tuning also the
 *           pixel-major copy of a chunk.
 */
int radon_fwd(const radon_op *op, const void *x, void *y, int32_t batch, int32_t layout,
              void *ws, int64_t ws_bytes, void *stream);

/*
 * radon_fwd_xt -- y = M R x when the caller already holds the transposed
 * images xT[b][ix][iy] = x[b][iy][ix] (device [batch][n*n]; NULL allowed
 * only when no measured angle is closer to horizontal than vertical, see
 * radon_op_info).  This is the single kernel radon_fwd runs after its
 * transpose (for images below 1024 pixels; larger ones are banded there,
 * which this call, having no workspace, does not do); CG keeps the
 * transposed direction up to date itself.
 */
int radon_fwd_xt(const radon_op *op, const void *x, const void *xT, void *y, int32_t batch,
                 void *stream);

/*
 * radon_adj -- x = R^T M^T y (the adjoint in eq:KKT, eq:PD_resolve,
 * eq:SB_solve), through the stored transpose: each output pixel is one
 * sequential sum, no atomics.  y: batch sinograms of n_meas_rays -> x: batch
 * images of n*n, both in `layout`.
 *   ws  radon_workspace_bytes(op, RADON_WS_ADJ, batch) bytes
 *       (| RADON_WS_PIXEL_LAYOUT for a pixel-major call).  An image-major call
 *       may pass NULL (or fewer bytes): it then stages every sinogram of a
 *       chunk on its own, whatever adj_layout says.
 */
int radon_adj(const radon_op *op, const void *y, void *x, int32_t batch, int32_t layout,
              void *ws, int64_t ws_bytes, void *stream);

/*
 * normal_apply -- out = alpha R^T M^T M R x + lambda K^T K x + sigma x.
 * With sigma = 0 this is the operator of eq:KKT and eq:SB_solve; with
 * alpha <- tau*alpha, lambda = 0, sigma = 1 that of eq:PD_resolve (Section 2).
 * K is the forward-difference gradient with a zero last difference
 * (Neumann), so K^T K is the 5-point grid Laplacian with Neumann boundary.
 *   x, out   device, batch images in `layout`; out must not alias x.
 *   dot_out  optional device double[batch]: <x, out> per image (FP64 sum of
 *            exact FP64 products, fixed order); NULL to skip.
 *   ws       radon_workspace_bytes(op, RADON_WS_NORMAL, batch) bytes
 *            (| RADON_WS_PIXEL_LAYOUT for a pixel-major call).
 */
int normal_apply(const radon_op *op, double alpha, double lambda, double sigma,
                 const void *x, void *out, double *dot_out, int32_t batch, int32_t layout,
                 void *ws, int64_t ws_bytes, void *stream);

/*
 * normal_apply_noalloc -- normal_apply for callers that cannot allocate or
 * pass device memory for a workspace: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same operation, same
 * kernels and bitwise the same result as normal_apply; the workspace is a
 * fixed device array of RADON_NOALLOC_SCRATCH_BYTES inside the library, one
 * copy per GPU, held until the process ends.  The call allocates nothing
 * (no hipMalloc, no allocating library routine); its first call on a device
 * looks the array's address up (hipGetSymbolAddress) with that device
 * current.
 *   x, out, dot_out, batch, stream: as for normal_apply (image-major).
 * Errors: as normal_apply; RADON_EWORKSPACE when
 * radon_workspace_bytes(op, RADON_WS_NORMAL, batch) exceeds the fixed size
 * (nothing is enqueued then).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams, host threads or processes without ordering) race
 * on it and give wrong results.  Nothing in it needs clearing between calls.
 */
#define RADON_NOALLOC_SCRATCH_BYTES (64ll << 20)
int normal_apply_noalloc(const radon_op *op, double alpha, double lambda, double sigma,
                         const void *x, void *out, double *dot_out, int32_t batch, void *stream);

typedef struct {
    int32_t iterations;   /* iterations that changed x */
    int32_t breakdown;    /* 0, or k+1 if iteration k met <p, Ap> <= 0 or non-finite */
    double rho0;          /* ||r_0||^2 */
    double rho;           /* ||r||^2 after the last iteration */
} radon_cg_info;

/*
 * cg_solve -- conjugate gradients (Hestenes-Stiefel) on
 * A = alpha R^T M^T M R + lambda K^T K + sigma I, one independent solve per
 * image (Section 2: the systems have no closed form and are solved
 * iteratively).  Vectors in the operator dtype, the scalars rho, gamma,
 * alpha_k and beta_k in FP64 on the device.
 *   rhs      device, batch images in `layout`.
 *   x        device, batch images in `layout`: initial guess if x0_given,
 *            else zeroed; receives the iterate.  r_0 = rhs - A x_0.
 *   n_iter   iteration cap; rtol > 0 also stops once ||r|| <= rtol ||r_0||;
 *            a zero residual stops; <p, Ap> <= 0 or non-finite stops and is
 *            reported as a breakdown.
 *   info     optional device radon_cg_info[batch].
 *   ws       radon_workspace_bytes(op, RADON_WS_CG, batch) bytes
 *            (| RADON_WS_PIXEL_LAYOUT for a pixel-major call).
 */
int cg_solve(const radon_op *op, double alpha, double lambda, double sigma,
             const void *rhs, void *x, int32_t x0_given, int32_t batch, int32_t layout,
             int32_t n_iter, double rtol, void *ws, int64_t ws_bytes,
             radon_cg_info *info, void *stream);

#define RADON_SB_WARM   1   /* mu holds the starting image */
#define RADON_SB_RESUME 2   /* continue from the state held in ws by a previous call */

typedef struct {
    double alpha;         /* data weight (eq:objmin) */
    double lambda;        /* splitting weight; shrink threshold is 1/lambda */
    double tol;           /* > 0: stop once the Bregman update's L1 norm falls
                             below tol times the first update's */
    int32_t n_outer;      /* Bregman iterations */
    int32_t n_cg;         /* CG iterations per Bregman iteration (inexact solve) */
    int32_t flags;        /* RADON_SB_WARM | RADON_SB_RESUME */
    int32_t reserved;
} radon_sb_params;

typedef struct {
    int32_t outer;        /* Bregman iterations run (this call) */
    int32_t breakdowns;   /* inner CG solves that reported a breakdown */
    double upd_b_first;   /* ||b^1 - b^0||_1 of the first update of the run */
    double upd_b;         /* ||b^{k+1} - b^k||_1 of the last iteration */
    double upd_u;         /* ||u^{k+1} - u^k||_1 of the last iteration */
} radon_sb_info;

/*
 * split_bregman_tv -- anisotropic-TV split Bregman (Goldstein-Osher, the
 * method of Section 4) for min_u alpha/2 ||M R u - f||^2 + ||K u||_1:
 *   per Bregman iteration, n_cg CG steps on
 *     (alpha R^T M^T M R + lambda K^T K) u = alpha R^T M^T f + lambda K^T (d - b)
 *   (eq:SB_solve, read with K^* as the transpose and a plus sign), warm
 *   started from the previous u with the residual carried across iterations,
 *   then d = shrink(K u + b, 1/lambda), b <- b + K u - d.
 *   f       device, batch sinograms of n_meas_rays in `layout`.
 *   mu      device, batch images in `layout`; the start if RADON_SB_WARM,
 *           receives u (and is read again by a RADON_SB_RESUME call).
 *   layout  RADON_LAYOUT_IMAGE or RADON_LAYOUT_PIXEL.
 *   ws      radon_workspace_bytes(op, RADON_WS_SB, batch) bytes
 *           (| RADON_WS_PIXEL_LAYOUT for a pixel-major call); holds d, b
 *           and the residual (always image-major), so a later call with
 *           RADON_SB_RESUME continues, in either layout.
 *   info    optional device radon_sb_info[batch].
 */
int split_bregman_tv(const radon_op *op, const radon_sb_params *params, const void *f,
                     void *mu, int32_t batch, int32_t layout, void *ws, int64_t ws_bytes,
                     radon_sb_info *info, void *stream);

/*
 * Unrolled CG with reverse mode, for gradients through a fixed number of CG
 * iterations on A = alpha R^T M^T M R + lambda K^T K + sigma I (the resolvent
 * system eq:PD_resolve of Section 2 with alpha <- tau*alpha, lambda = 0,
 * sigma = 1; any SPD choice works).  x_n = CG_n(rhs) from x_0 = 0 is a
 * nonlinear function of rhs (the step lengths and the beta_k depend on it);
 * cg_unrolled_vjp returns (d x_n / d rhs)^T gx exactly for the iterations the
 * forward ran, by reverse-mode differentiation of each Hestenes-Stiefel
 * update.  The forward keeps (r, p, rho) every `ckpt` iterations in a tape;
 * the reverse replays each ckpt-long segment from its checkpoint with the
 * same kernels (bitwise the forward's iterates) before sweeping back through
 * it, so memory is n_iter/ckpt checkpoints plus one segment of records.
 * An iteration that stopped (rho == 0 or a breakdown) passes the adjoints
 * through unchanged.
 *
 * radon_unrolled_sizes -- bytes of the tape (tape_bytes), of the forward's
 * workspace (ws_fwd_bytes) and of the reverse's workspace (ws_vjp_bytes) for
 * these sizes; each pointer may be NULL.
 */
int radon_unrolled_sizes(const radon_op *op, int32_t n_iter, int32_t ckpt, int32_t batch,
                         int64_t *tape_bytes, int64_t *ws_fwd_bytes, int64_t *ws_vjp_bytes);

/*
 * cg_unrolled -- x = CG_n(rhs) from x_0 = 0, no tolerance stop; writes the tape.
 *   rhs, x  device [batch][n*n], operator dtype; x must not alias rhs.
 *   tape    device, tape_bytes >= radon_unrolled_sizes' tape_bytes; owned by
 *           the caller, read by cg_unrolled_vjp with the same op, alpha,
 *           lambda, sigma, batch, n_iter and ckpt.
 *   ws      device, radon_unrolled_sizes' ws_fwd_bytes; scratch.
 */
int cg_unrolled(const radon_op *op, double alpha, double lambda, double sigma,
                const void *rhs, void *x, int32_t batch, int32_t n_iter, int32_t ckpt,
                void *tape, int64_t tape_bytes, void *ws, int64_t ws_bytes, void *stream);

/*
 * cg_unrolled_vjp -- grhs = (d x_n / d rhs)^T gx for the solve cg_unrolled
 * recorded in `tape` (rhs itself is the tape's first checkpoint).
 *   gx      device [batch][n*n]: dL/dx_n.
 *   grhs    device [batch][n*n]: dL/drhs, written; may alias gx.
 *   ws      device, radon_unrolled_sizes' ws_vjp_bytes; scratch.
 * Errors: RADON_EWORKSPACE for a short tape or workspace, RADON_EINVAL for
 * n_iter < 0, ckpt < 1 or NULL vectors.
 */
int cg_unrolled_vjp(const radon_op *op, double alpha, double lambda, double sigma,
                    const void *tape, int64_t tape_bytes, const void *gx, void *grhs,
                    int32_t batch, int32_t n_iter, int32_t ckpt, void *ws, int64_t ws_bytes,
                    void *stream);

/*
 * Mixed batches: several operators of different geometry (image size, angle
 * and bin counts) in one group, so that each phase of a product or of a CG
 * iteration is a single launch over all instances instead of one launch per
 * instance.  The instance count, sizes and weights are fixed at creation.
 *
 * Packed vectors: instance i's image occupies elements
 * [img_off[i], img_off[i] + n_i*n_i) of one device vector of img_off[count]
 * elements (operator dtype), its measured sinogram
 * [sino_off[i], sino_off[i] + n_meas_rays_i) of one vector of
 * sino_off[count]; each start is 256-byte aligned and the gaps are ignored.
 */
typedef struct radon_multi radon_multi;   /* opaque group handle */
typedef struct radon_graph radon_graph;   /* opaque captured-graph handle */

/*
 * radon_multi_create -- group `count` operators (all of one dtype and one
 * forward bundle width).  The
 * group borrows the operators: they must outlive it.  alpha, lambda, sigma:
 * host arrays of `count` weights of each instance's normal operator
 * A_i = alpha_i R_i^T M_i^T M_i R_i + lambda_i K^T K + sigma_i I (Section 2),
 * or NULL for 1, 0, 0.  Synchronous (copies the work lists to the device).
 */
int radon_multi_create(const radon_op *const *ops, int32_t count, const double *alpha,
                       const double *lambda, const double *sigma, radon_multi **out);

/*
 * The group with its device tables in caller storage: radon_multi_table_bytes
 * reports the bytes of the group's tables (instance descriptors, the
 * concatenated forward work list, instance start tables; synchronous, it
 * reads the operators' work orders), and radon_multi_create_into builds the
 * group as radon_multi_create does, into `tables` (device, 256-byte aligned,
 * at least that many bytes, owned by the caller and kept alive and untouched
 * while the group lives).  The handle then owns no device memory.
 * Errors: as radon_multi_create; RADON_EWORKSPACE for too few bytes.
 */
int radon_multi_table_bytes(const radon_op *const *ops, int32_t count, int64_t *bytes);
int radon_multi_create_into(const radon_op *const *ops, int32_t count, const double *alpha,
                            const double *lambda, const double *sigma, void *tables,
                            int64_t tables_bytes, radon_multi **out);
void radon_multi_destroy(radon_multi *m);

/*
 * radon_multi_info -- packed-vector offsets (host int64[count+1] each, NULL
 * to skip), workspace bytes of radon_multi_apply and radon_multi_cg, and the
 * waves per ray bundle and per 8x8 tile the group's products use (a single
 * operator tuned to the same counts computes bitwise the same products).
 */
int radon_multi_info(const radon_multi *m, int64_t *img_off, int64_t *sino_off,
                     int64_t *ws_products, int64_t *ws_cg, int32_t *fwd_waves,
                     int32_t *adj_waves);

/*
 * radon_multi_apply -- which = 0: y_i = M_i R_i x_i (in: packed images, out:
 * packed sinograms); 1: x_i = R_i^T M_i^T y_i (packed sinograms -> images);
 * 2: out_i = A_i x_i (packed images -> images).  ws: ws_products bytes.
 */
int radon_multi_apply(const radon_multi *m, int32_t which, const void *in, void *out,
                      void *ws, int64_t ws_bytes, void *stream);

/*
 * radon_multi_cg -- CG (Hestenes-Stiefel) on A_i x_i = rhs_i from x_i = 0,
 * one independent solve per instance with FP64 scalars (as cg_solve).
 *   rhs, x  packed images; x must not alias rhs.
 *   info    optional device radon_cg_info[count].
 *   ws      ws_cg bytes.
 */
int radon_multi_cg(const radon_multi *m, const void *rhs, void *x, int32_t n_iter, double rtol,
                   void *ws, int64_t ws_bytes, radon_cg_info *info, void *stream);

/*
 * radon_multi_cg_graph -- capture the radon_multi_cg call with these
 * arguments into a HIP graph (nothing runs yet).  Each radon_graph_launch
 * then runs the whole solve with one launch, reading rhs and writing x, info
 * and ws at the captured addresses: those buffers, the group and its
 * operators must stay alive while the graph exists.  The graph holds no
 * memset nodes.  Replays on one stream run in order; replays that overlap
 * (other streams) race on the captured buffers.
 */
int radon_multi_cg_graph(const radon_multi *m, const void *rhs, void *x, int32_t n_iter,
                         double rtol, void *ws, int64_t ws_bytes, radon_cg_info *info,
                         radon_graph **out);
int radon_graph_launch(const radon_graph *g, void *stream);
void radon_graph_destroy(radon_graph *g);

/*
 * chambolle_pock_tv -- the primal-dual method of Chambolle and Pock, whose
 * primal step is the resolvent system eq:PD_resolve (Section 2), for
 * min_u ||K u||_1 + alpha/2 ||M R u - f||^2 (anisotropic TV):
 *   y <- clip(y + sigma K ubar, -1, 1);
 *   u_new: n_cg CG steps on (I + tau alpha R^T M^T M R) u_new
 *          = u - tau K^T y + tau alpha R^T M^T f, from u_new = u with its true
 *          residual;
 *   ubar <- 2 u_new - u.
 * y starts at 0, ubar at u; convergence needs tau sigma ||K||^2 < 1, and
 * ||K||^2 <= 8.  Each outer step costs n_cg + 1 normal-operator applies.
 *   f   device [batch][n_meas_rays];  mu device [batch][n*n]: the start if
 *       flags has RADON_SB_WARM (else zeroed), receives u.
 *   ws  radon_workspace_bytes(op, RADON_WS_PD, batch) bytes.
 */
typedef struct {
    double alpha;         /* data weight (eq:objmin) */
    double tau, sigma;    /* primal and dual step sizes */
    int32_t n_outer;      /* primal-dual iterations */
    int32_t n_cg;         /* CG steps per resolvent solve */
    int32_t flags;        /* RADON_SB_WARM */
    int32_t reserved;
} radon_pd_params;

int chambolle_pock_tv(const radon_op *op, const radon_pd_params *params, const void *f,
                      void *mu, int32_t batch, void *ws, int64_t ws_bytes, void *stream);

/*
 * Surrogate operator T (Section 3.2, eq:def_sparse_surr): the sum over all
 * pixels q of the point-spread function P = R^T M^T M R e_c of the centre
 * pixel c = (n/2, n/2) (0-based), moved to q and cut to the disc |d| <= r
 * around q, entries outside the image dropped (no wrap-around).  T is taken
 * as the symmetric part of that sum: weight w(d) = (P_{c+d} + P_{c-d}) / 2
 * for |d| <= r, so (T x)_p = sum_d w(d) x_{p-d} over taps inside the image.
 * It replaces R^T M^T M R in the split-Bregman update (eq:surr_SBupd), where
 * the data right-hand side keeps the exact adjoint.
 */
typedef struct radon_surrogate radon_surrogate;   /* opaque surrogate handle */

/*
 * radon_surrogate_create -- build T of radius r (0 <= r <= 8; the disc must
 * fit in the image) from `op`'s own products.  Synchronous on `stream`.  The
 * handle owns its weights (device and host) and does not borrow `op`.
 */
int radon_surrogate_create(const radon_op *op, int32_t radius, void *stream,
                           radon_surrogate **out);
void radon_surrogate_destroy(radon_surrogate *s);

/* radon_surrogate_weights -- radius, and the (2r+1)^2 weights (host double,
 * row-major in (dy, dx), zero outside the disc); either pointer may be NULL. */
int radon_surrogate_weights(const radon_surrogate *s, int32_t *radius, double *w);

/*
 * surrogate_apply -- out = alpha T x + lambda K^T K x + sigma x (x, out
 * device [batch][n*n] in the operator dtype, out must not alias x); with
 * dot_out (device double[batch]) also <x, out> per image, which needs a
 * workspace ws of 8 * ceil(n/32)^2 * batch bytes (none otherwise).
 */
int surrogate_apply(const radon_surrogate *s, double alpha, double lambda, double sigma,
                    const void *x, void *out, double *dot_out, int32_t batch, void *ws,
                    int64_t ws_bytes, void *stream);

/*
 * split_bregman_tv_surrogate -- split_bregman_tv with every inner CG solve
 * on alpha T + lambda K^T K (eq:surr_SBupd) instead of the exact normal
 * operator; the data term alpha (MR)^T f, the shrink and Bregman steps and
 * the workspace (RADON_WS_SB) are those of split_bregman_tv.  A run with
 * RADON_SB_WARM can start the exact solver from its result.
 */
int split_bregman_tv_surrogate(const radon_op *op, const radon_surrogate *s,
                               const radon_sb_params *params, const void *f, void *mu,
                               int32_t batch, void *ws, int64_t ws_bytes, radon_sb_info *info,
                               void *stream);

/*
 * split_bregman_tv_graph -- split_bregman_tv (exact operator) captured once
 * as a HIP graph: every kernel of the n_outer x n_cg solve becomes one node,
 * so a reconstruction is one radon_graph_launch with no host work between
 * kernels.  Each launch reads f and writes mu, ws and info at the addresses
 * given here, and runs the whole solve from the start (from mu with
 * RADON_SB_WARM, else from 0); RADON_SB_RESUME cannot be captured.  The
 * buffers must stay allocated while the graph is used.  Release with
 * radon_graph_destroy.  Arguments and errors as for split_bregman_tv.
 */
int split_bregman_tv_graph(const radon_op *op, const radon_sb_params *params, const void *f,
                           void *mu, int32_t batch, void *ws, int64_t ws_bytes, radon_sb_info *info,
                           radon_graph **out);

/*
 * Fourier-domain operator (Sections 2 and 3.1: eq:four_obj, eq:SBFFT,
 * eq:fusedop).  By the Fourier slice theorem, the 1-D DFT of the projection
 * at measured angle theta_k = pi k / n_angles and radial frequency
 * rho_q = 2 pi q / n_bins samples the 2-D Fourier transform of the image at
 *   xi_p = rho_q (cos theta_k, sin theta_k),  q = -Q .. Q,  Q = (n_bins-1)/2
 * (integer division, so the set is closed under xi -> -xi).  Point p =
 * a (2Q + 1) + q + Q for the a-th measured angle.  With pixel modes
 * m = (ix - n/2, iy - n/2) (integer division) the forward map is
 *   (F^* mu)_p = sum_m mu_m exp(-i xi_p . m),
 * its adjoint (F fhat)_m = sum_p fhat_p exp(+i xi_p . m), and the split-
 * Bregman system eq:SBFFT needs H = Re(F F^*).  All three are evaluated by
 * Gaussian gridding (the NUFFT of Greengard and Lee) on an M x M frequency
 * grid (M a power of two, 2n <= M <= 4096), with the heat kernel
 * exp(-|xi - eta|^2 / (4 tau)) over the 2 m_sp nearest grid points per
 * dimension and the deconvolution A = (pi / tau) exp(|m|^2 tau):
 *   F^* ~ B^* F_D^* A,   F ~ A F_D B,
 *   H   ~ Re(A F_D (B B^*) F_D^* A)   with B B^* precomputed as one sparse
 *         grid-to-grid matrix (RADON_FOURIER_FUSED, eq:fusedop), or as the
 *         product of the two gridded transforms (RADON_FOURIER_NUFFT).
 * Complex arrays are interleaved (re, im) pairs of the operator's vector type
 * (float for SPARSECT_F32, double otherwise); the stored gridding weights and
 * B B^* use the matrix value type.  The handle borrows `op` (which must
 * outlive it) and owns its tables.
 */
typedef struct radon_fourier radon_fourier;   /* opaque Fourier-operator handle */

typedef struct {
    int64_t n_points;       /* P = n_meas_angles * (2Q + 1) */
    int32_t grid;           /* M */
    int32_t m_sp;           /* half window, grid points per dimension */
    double tau;             /* heat-kernel width */
    int64_t fused_tiles;    /* stored 8 x 8 grid tiles of B B^* (the others are zero) */
    int64_t fused_bytes;    /* bytes of their coefficients */
    int64_t spread_nnz;     /* entries of the gridding matrix B: P (2 m_sp)^2 */
    int64_t device_bytes;   /* device memory held by the handle */
} radon_fourier_info;

#define RADON_FOURIER_FUSED 0   /* H through the precomputed B B^* */
#define RADON_FOURIER_NUFFT 1   /* H as the gridded F composed with the gridded F^* */

#define RADON_FWS_TRANSFORM 0   /* fourier_fwd, fourier_adj, fourier_normal */
#define RADON_FWS_SB        1   /* split_bregman_tv_fourier */

/*
 * radon_fourier_create -- point set, gridding tables and B B^* of `op`'s
 * geometry.  m_sp in [1, 12] (6 and 12 give about 6 and 12 digits); tau 0
 * selects 4 m_sp / M^2 (= m_sp / n^2 on the 2n grid); grid 0 selects the
 * smallest power of two >= 2n.  B B^* is stored as a variable-coefficient
 * stencil: for each grid point s of a non-empty 8 x 8 tile, its
 * (4 m_sp - 1)^2 coefficients C[s][d] = sum_p g_p(s) g_p(s + d) (periodic
 * indices).  Synchronous on `stream`; the handle owns all its device memory.
 */
int radon_fourier_create(const radon_op *op, int32_t m_sp, double tau, int32_t grid, void *stream,
                         radon_fourier **out);
void radon_fourier_destroy(radon_fourier *f);
int radon_fourier_get_info(const radon_fourier *f, radon_fourier_info *out);
/* workspace bytes for `which` (RADON_FWS_*) and `batch` images; -1 on error */
int64_t radon_fourier_workspace_bytes(const radon_fourier *f, int32_t which, int32_t batch);

/*
 * fourier_fwd -- fhat = F^* mu (gridded): mu device [batch][n*n], fhat device
 * [batch][P] complex.  ws: radon_fourier_workspace_bytes(RADON_FWS_TRANSFORM);
 * errors and stream as for fourier_normal.
 */
int fourier_fwd(const radon_fourier *f, const void *mu, void *fhat, int32_t batch, void *ws,
                int64_t ws_bytes, void *stream);

/*
 * fourier_adj -- x = alpha Re(F fhat) (gridded): fhat device [batch][P]
 * complex, x device [batch][n*n].  This is the data term of eq:SBFFT.
 * ws, errors and stream as for fourier_normal.
 */
int fourier_adj(const radon_fourier *f, const void *fhat, void *x, double alpha, int32_t batch,
                void *ws, int64_t ws_bytes, void *stream);

/*
 * fourier_normal -- out = alpha H x + lambda K^T K x + sigma x with H by
 * `path` (RADON_FOURIER_FUSED or RADON_FOURIER_NUFFT); with dot_out (device
 * double[batch]) also <x, out>.  x, out device [batch][n*n]; out must not
 * alias x.  ws: radon_fourier_workspace_bytes(RADON_FWS_TRANSFORM) (two
 * M x M complex grids and the sample values per image).  Errors: EINVAL for
 * a NULL handle or pointer, an unknown path, aliasing or a short workspace;
 * EUNSUPPORTED for batch > 65535.  Asynchronous on `stream`.
 */
int fourier_normal(const radon_fourier *f, int32_t path, double alpha, double lambda, double sigma,
                   const void *x, void *out, double *dot_out, int32_t batch, void *ws,
                   int64_t ws_bytes, void *stream);

/*
 * split_bregman_tv_fourier -- split_bregman_tv on eq:SBFFT: every inner CG
 * solve is on alpha H + lambda K^T K (H by `path`), the data term is
 * alpha Re(F fhat) with fhat device [batch][P] complex; params, mu and info
 * as for split_bregman_tv.  ws: radon_fourier_workspace_bytes(RADON_FWS_SB).
 */
int split_bregman_tv_fourier(const radon_fourier *f, int32_t path, const radon_sb_params *params,
                             const void *fhat, void *mu, int32_t batch, void *ws, int64_t ws_bytes,
                             radon_sb_info *info, void *stream);

/*
 * Launch tuning of an operator (not part of the method: it only changes how
 * the products are scheduled; the waves-per-item counts, the band height and
 * the gather layout split each sum differently, so results change at the
 * rounding level).
 *   fwd_waves  waves per ray bundle in the forward product: 2 or 4;
 *   adj_waves  waves per 8x8 tile in the adjoint: 1, 2 or 4 (0: chosen from
 *              the number of measured angles, or of stored angles for an
 *              adjoint stored by symmetry);
 *   fwd_rhs, adj_rhs  largest number of images (right-hand sides) that share
 *              each matrix load in a fused multi-image product: 1, 4, 8, 16;
 *   fwd_layout how a fused forward chunk of 4 or more images gathers its
 *              pixels: 0 = from each image in turn; 1 = from a pixel-major
 *              copy of the chunk (a pixel's values for all images of the
 *              chunk contiguous, so one 16-byte load serves 4 FP32 or 2 FP64
 *              images), made in the call's workspace;
 *   adj_layout how a fused adjoint chunk of 4 or more sinograms stages its
 *              bands: 0 = from each sinogram in turn; 1 = from a pixel-major
 *              copy of the chunk's sinograms (a measurement's values for all
 *              images contiguous), made in the call's workspace (radon_adj
 *              uses it only when given a workspace of the size
 *              radon_workspace_bytes reports).  For an adjoint stored by
 *              symmetry (radon_info.adj_symmetric), whatever the image count:
 *              0 = one workgroup per 8x8 tile (adj_waves waves), 1 = one
 *              workgroup per orbit of tiles under the maps, reading each
 *              stored slot once (2 x adj_waves waves, 8 for 0; radon_autotune
 *              tries it from 1024 orbits on);
 *   fwd_lines  height of the line bands of a forward that has a workspace:
 *              0 = chosen from the chunk's image bytes (the largest of 128,
 *              64, 32, 16 lines whose band of the chunk's images fits 2 MB;
 *              none below 1024 pixels while the chunk's whole images fit);
 *              16, 32, 64 or 128 = that height (operators from 256 pixels
 *              on; smaller ones accept only 0).
 * The workspace sizes of radon_workspace_bytes depend on the tuning at the
 * time of the query.  radon_set_tuning must not overlap with enqueued work on
 * the operator.  radon_autotune times the candidates and caches the best per
 * geometry.
 */
typedef struct {
    int32_t fwd_waves, adj_waves, fwd_rhs, adj_rhs, fwd_layout, fwd_lines, adj_layout;
    int32_t reserved;   /* 0 */
} radon_tuning;

int radon_set_tuning(radon_op *op, const radon_tuning *t);
int radon_get_tuning(const radon_op *op, radon_tuning *out);

/*
 * radon_autotune -- choose op's radon_tuning by timing the candidates on its
 * own geometry (HIP events on `stream`): waves per forward bundle (2, 4) and
 * per adjoint tile (1, 2, 4) on one image, one knob at a time; then, for
 * batch > 1, the images sharing each matrix load in the forward and in the
 * adjoint (1, 4, 8, 16 each; at most batch), jointly on the normal
 * operator's two products; then, at that adjoint chunk, every forward chunk
 * of 4 or more images with each gather layout (fwd_layout) and band height
 * (fwd_lines) the operator has, and the adjoint chunk's staging layout
 * (adj_layout).  The search starts from fwd_layout = adj_layout = 0 and
 * fwd_lines = 0.  The forward bundle width is a layout choice made at build
 * time (radon_geom.fwd_bundle), not tuned here.
 *   batch       the batch the operator will run at (1 .. 65535).
 *   ws          device, radon_workspace_bytes(op, RADON_WS_TUNE, batch) bytes
 *               (test images and products; the values do not matter); may
 *               be NULL with RADON_TUNE_CACHED_ONLY.
 *   cache_path  NULL, or a text file of earlier results keyed by GPU
 *               architecture, geometry, measured angles, dtype, bundle width
 *               and batch: an entry found there is applied without timing;
 *               a timed result is appended.
 *   flags       RADON_TUNE_CACHED_ONLY: apply a cached entry if there is one,
 *               never time (the tuning stays as it was otherwise).
 *   source      optional host int: 0 = unchanged, 1 = from the cache,
 *               2 = timed now.
 * Synchronises `stream` when it times.  Must not overlap with other work on
 * the operator.  Errors: RADON_EWORKSPACE, RADON_EINVAL (bad flags, a cache
 * that cannot be written), RADON_EHIP.
 */
#define RADON_TUNE_CACHED_ONLY 1
int radon_autotune(radon_op *op, int32_t batch, void *ws, int64_t ws_bytes, const char *cache_path,
                   int32_t flags, void *stream, int32_t *source);

/*
 * radon_bandwidth_probe -- the practical HBM ceiling the products are
 * measured against (not part of the method).  RADON_PROBE_COPY: dst = src
 * (bytes read + bytes written); RADON_PROBE_READ: a read-only pass over src
 * that leaves one 32-bit xor-sum per workgroup in dst (dst holds 4096 uint32).
 * Both stream with 16-byte non-temporal loads (the copy grid-stride over 8192
 * workgroups, the read one contiguous chunk per workgroup over 4096).
 * src, dst: device, 16-byte aligned; bytes: positive multiple of 16.
 * Asynchronous on `stream`.  Errors: RADON_EINVAL.
 */
#define RADON_PROBE_COPY 0
#define RADON_PROBE_READ 1
int radon_bandwidth_probe(int32_t mode, const void *src, void *dst, int64_t bytes, void *stream);

/*
 * radon_export_csr -- copy the CSR of MR to host memory (synchronous; for
 * checks and external tools).  row_ptr int64[n_meas_rays+1], col int32[nnz],
 * val double[nnz] (entries widened from the operator dtype), each NULL to
 * skip.  Entries are in the order the ray visits the pixels.
 */
int radon_export_csr(const radon_op *op, int64_t *row_ptr, int32_t *col, double *val);

/*
 * radon_export_adj -- copy the pixel-group layout of (MR)^T to host memory as
 * per-(pixel, measured angle) records: bin int32[n*n*n_meas_angles] (first
 * bin, or -1 if no ray of that angle crosses the pixel), v0 and v1
 * double[n*n*n_meas_angles] (lengths for that bin and the next one).  Record
 * (j, a) is at j*n_meas_angles + a.  A layout stored by symmetry is read
 * through its maps, so every measured angle has its records.  Synchronous.
 */
int radon_export_adj(const radon_op *op, int32_t *bin, double *v0, double *v1);

#ifdef __cplusplus
}
#endif

#endif /* SPARSECT_H */
