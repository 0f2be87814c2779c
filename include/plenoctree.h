/*
 * plenoctree.h -- C ABI of libplenoctree.so, an MI355X (gfx950) renderer for
 * PlenOctrees (Yu et al., "PlenOctrees for Real-time Rendering of Neural
 * Radiance Fields", ICCV 2021, arXiv 2103.14024).
 *
 * A PlenOctree is a sparse octree over an axis-aligned box whose data leaves
 * hold a raw density and, for each RGB channel, a vector of real spherical
 * harmonic (SH) coefficients (Sec. 4.2, "Sampling"; SH of App. B.1).  A ray
 * is cut into the exact segments between voxel boundaries, large empty voxels
 * being crossed in one step (Sec. 4.2, "Rendering"); each data segment
 * contributes with the piecewise-constant quadrature of Sec. 3 (eqn:quad) and
 * the background term of App. B.3; marching stops early once the
 * transmittance falls below a threshold (Sec. 4.2, "Rendering").  The
 * gradient entry point implements the analytic derivatives of App. B.3 for
 * the direct optimisation of Sec. 4.3.
 *
 * General conventions
 *  - Every function returns a po_status.  On any code other than PO_OK the
 *    call has written no output and queued no GPU work; po_last_error()
 *    returns a message for the calling thread.  No C++ exception crosses the
 *    ABI.
 *  - "d_" pointers are device pointers (HBM of the current HIP device),
 *    "h_" / plain pointers are host pointers.  The caller owns every buffer.
 *    A po_tree handle owns only its metadata and borrows the device arrays
 *    given to po_tree_bind; they must outlive all work queued with it.
 *  - Render calls only enqueue work on `stream` (a hipStream_t; NULL is the
 *    null stream) and return; outputs are valid once the stream has
 *    completed.  Handles are immutable after bind, so renders of one tree on
 *    several streams may run concurrently.
 *  - n == 0 (no rays) is a no-op returning PO_OK.
 *
 * Geometry
 *  - The tree box is [center - half_size, center + half_size]^3 in world
 *    units.  Level 0 is the box; a cell at level L has edge
 *    2*half_size / 2^L and integer coordinates (i, j, k) in [0, 2^L)^3.
 *  - Child array: int32 child[n_nodes][8]; node 0 is the root.  The child
 *    slot of a cell is 4*xbit + 2*ybit + zbit (bits of the child's integer
 *    coordinates).  Entry e > 0: internal node e.  e == 0: empty space
 *    (density 0, no record).  e < 0: data leaf number -e-1.
 *  - Leaf records: sigma[n_leaves] (raw density; the renderer uses
 *    max(sigma, 0), App. B.3 last paragraph) and sh[n_leaves][sh_stride],
 *    whose first 3*K elements are channel-major coefficients
 *    sh[leaf][c*K + l*l + l + m], K = (sh_degree+1)^2 (Sec. 4.1).  Both
 *    arrays are float32 (PO_F32) or IEEE binary16 (PO_F16); FP16 values are
 *    widened to float32 and all arithmetic is float32.
 *  - Rays: origins o and directions d, float32 [n][3]; d need not be unit
 *    length (it is normalised; segment lengths are world units along the
 *    unit direction).  A ray starts at t = 0 (origins inside the box render
 *    from the origin).  The SH basis is evaluated at the unit direction of
 *    propagation.
 *  - Camera: pinhole through pixel centres; pixel (row v, column u) looks
 *    along R * ((u + 0.5 - cx)/fx, -(v + 0.5 - cy)/fy, -1), R the first three
 *    columns of the row-major 3x4 camera-to-world matrix c2w whose last
 *    column is the camera position (OpenGL frame: -z forward, +y up).
 *    Images are row-major [height][width][3] float32.
 */
#ifndef PLENOCTREE_H
#define PLENOCTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PO_MAX_DEPTH 15
#define PO_MAX_SH_DEGREE 4
#define PO_BATCH_MAX_JOBS 16
#define PO_TILE 16 /* camera images are processed in 16 x 16 pixel tiles */

typedef enum {
    PO_OK = 0,
    PO_ERR_INVALID = 1,     /* bad argument: NULL pointer, negative size, bad option, misalignment */
    PO_ERR_TREE = 2,        /* malformed tree or cell list */
    PO_ERR_OOM = 3,         /* host allocation failed */
    PO_ERR_DEVICE = 4,      /* HIP runtime error */
    PO_ERR_UNSUPPORTED = 5  /* valid but unsupported combination */
} po_status;

typedef enum { PO_F32 = 0, PO_F16 = 1 } po_dtype;

/* Description of a tree.  sh_stride: elements from one leaf's SH record to
 * the next; 0 means 3*K.  Must be >= 3*K, and sh_stride * element size must
 * be a multiple of 4 bytes. */
typedef struct {
    int32_t depth;      /* maximum depth D, 1..PO_MAX_DEPTH */
    int32_t sh_degree;  /* l_max, 0..PO_MAX_SH_DEGREE */
    float center[3];
    float half_size;    /* > 0 */
    int32_t dtype;      /* po_dtype of sigma and sh */
    int32_t sh_stride;
} po_tree_desc;

/* Per-call rendering options.
 *
 * PO_OUT_AUX also writes aux[ray][4] = {final transmittance T, data samples,
 * traversal steps, depth}.  1 - T is the alpha map.  depth is the expected
 * termination distance of the viewer's depth map (Sec. 5.5): the sum over the
 * composited data segments [a, b] of the integral of t sigma T(t) dt, with t
 * the distance from the ray origin in world units; it is not normalised by
 * the opacity (divide by 1 - T for the mean over the opaque part).
 *
 * sh_off and clip are the other viewer options of Sec. 5.5.  Bit k of sh_off
 * drops SH basis function k (index l*l + l + m) from every channel, so the
 * colour of a leaf is the sigmoid of the remaining terms; bits at or above K
 * have no effect.  clip = (nx, ny, nz, w) is a slicing plane: only the part
 * of each ray where nx*x + ny*y + nz*z + w >= 0 is rendered (all zero: the
 * whole ray).  These options apply to rendering only; the backward pass
 * rejects them.  A call that sets none of them and no PO_OUT_AUX runs the
 * plain kernels. */
#define PO_OUT_AUX 1u
/* PO_ONE_PASS: walk every ray to its end in one pass by one lane, also where
 * po_render_camera, po_render_rays or po_render_batch would render in pieces
 * (the reference of the split render's equality, and for timing it). */
#define PO_ONE_PASS 2u
typedef struct {
    float bg[3];        /* background colour c_N (App. B.3) */
    float stop_T;       /* early stop once T < stop_T after a data segment (Sec. 4.2); 0 disables */
    int32_t max_steps;  /* cap on traversal steps per ray; 0 = 3*2^D + 8, which valid trees never reach */
    uint32_t flags;     /* PO_OUT_AUX | PO_ONE_PASS */
    uint32_t sh_off;    /* SH basis functions left out (bit k = function k); 0 = none */
    float clip[4];      /* slicing half-space n.x + w >= 0; all zero = none */
} po_render_opts;

typedef struct {
    float c2w[12];      /* row-major 3x4 camera-to-world */
    int32_t width, height;
    float fx, fy, cx, cy;
} po_camera;

typedef struct po_tree po_tree;       /* opaque, immutable after bind */
typedef struct po_builder po_builder; /* opaque, host-side build state */

/* ------------------------------------------------------------------ build
 * Octree construction from leaf cells (Sec. 4.2, "Filtering": the surviving
 * voxels become leaves, everything else is empty).  Host only, no GPU.
 *
 * po_builder_create: h_cells is [n_cells][4] int32 (level, i, j, k) with
 * 1 <= level <= depth and coordinates in [0, 2^level).  Cells must not
 * overlap.  Leaves are numbered in Morton order of their corner; internal
 * nodes are numbered level by level (all nodes of level L before any of level
 * L+1), Morton order within a level, so the top levels form a prefix of the
 * child array.  Errors: PO_ERR_INVALID (NULL, n_cells < 0, bad desc),
 * PO_ERR_TREE (cell out of range, overlapping or duplicate cells),
 * PO_ERR_OOM. */
po_status po_builder_create(const po_tree_desc* desc, int64_t n_cells, const int32_t* h_cells,
                            po_builder** out);
/* Sizes of the built tree: n_nodes (>= 1, the root always exists) and n_leaves (== n_cells). */
po_status po_builder_sizes(const po_builder* b, int64_t* n_nodes, int64_t* n_leaves);
/* Writes h_child[n_nodes][8] and h_leaf_perm[n_leaves]: leaf j of the tree is
 * the caller's cell h_leaf_perm[j] (so sigma_tree[j] = sigma_cells[perm[j]]). */
po_status po_builder_emit(const po_builder* b, int32_t* h_child, int64_t* h_leaf_perm);
po_status po_builder_destroy(po_builder* b);

/* Checks a host copy of a child array: every entry in range, every internal
 * node referenced exactly once and reachable from the root (no cycles, no
 * sharing), no internal node at depth D, and, when h_sigma is not NULL
 * (dtype of desc, n_leaves values), every density finite.  PO_ERR_TREE with
 * a message naming the first fault. */
po_status po_tree_validate(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child,
                           int64_t n_leaves, const void* h_sigma);

/* -------------------------------------------------------------------- bind
 * Wraps device arrays (child, sigma, sh as described above) in a handle.  No
 * data is copied or checked on the device (po_tree_build_index, called once
 * after binding, adds the traversal index that speeds up the walk; without
 * it the kernels walk the caller's child array); the kernels treat an out-of-range
 * entry, or an internal node below depth D, as empty space and count it in
 * the device error counter (po_device_errors), so a malformed array cannot
 * make them read out of bounds.  d_sh must be aligned to 4 bytes (16 for the
 * fastest loads).  Each of the three arrays must be smaller than 4 GiB - 256
 * bytes (the kernels address them with 32-bit buffer offsets); larger trees
 * return PO_ERR_UNSUPPORTED.  Errors: PO_ERR_INVALID, PO_ERR_UNSUPPORTED. */
po_status po_tree_bind(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child,
                       int64_t n_leaves, const void* d_sigma, const void* d_sh, po_tree** out);
/* po_tree_bind_sg: as po_tree_bind, for a tree whose colour basis is
 * K = (sh_degree+1)^2 spherical Gaussians instead of the SH (App. B.1, the
 * SG-25 variant of the basis ablation, App. A): the colour of a leaf is
 * sigmoid(sum_j k_j G_j(d)) with G_j(d) = exp(lambda_j (d . p_j / |p_j| -
 * 1)).  d_lobes is a device array [K][4] = (p_x, p_y, p_z, lambda) of the
 * lobes shared by all leaves, float32, 16-byte aligned, borrowed like the
 * other arrays; every axis must be non-zero.  The leaf records keep the SH
 * layout with K coefficients per channel.  Renders, gradients (with respect
 * to the leaf values; the lobes are held fixed) and the filter all use the
 * bound basis; sh_off then drops lobes.  Errors as for po_tree_bind. */
po_status po_tree_bind_sg(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child, int64_t n_leaves,
                          const void* d_sigma, const void* d_sh, const float* d_lobes, po_tree** out);
/* po_tree_bind_codebook: binds a tree whose leaf colours are compressed
 * with per-basis-function codebooks (App. B.2; build them with
 * po_codebook_build).  desc->dtype must be PO_F16: d_sigma holds the float16
 * densities.  d_index [n_leaves][stride] uint16 replaces the SH records:
 * entry k is the leaf's codebook position for basis function k (stride =
 * desc->sh_stride, even and >= K; 0 means K rounded up to a multiple of 4).
 * d_codebook [K][M][4] float16, 8-byte aligned: (r, g, b, unused) per entry.
 * The colour of a leaf is that of an SH leaf with coefficient (c, k) =
 * codebook[k][index[k]][c].  Camera, ray and batched renders and the
 * visibility filter accept codebook trees (no aux outputs, sh_off or slicing
 * plane); gradients do not.  An index >= M reads another basis function's
 * entry, or zero past the end of the codebook.  Errors as for po_tree_bind. */
po_status po_tree_bind_codebook(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child, int64_t n_leaves,
                                const void* d_sigma, const uint16_t* d_index, const void* d_codebook, int32_t M,
                                po_tree** out);
/* po_tree_build_index: builds the handle's traversal index, a derived copy
 * of the child array that the renders, gradients and the filter walk
 * instead of the caller's array.  The nodes above level M = D - 3 keep
 * their child entries; each internal node of level M becomes a brick of
 * 8 x 8 x 8 entries, one per finest cell of its cube, naming the leaf (or
 * empty space) that holds the cell and that leaf's level.  A walk step
 * inside one brick then needs one dependent read instead of one per level
 * below the common ancestor; the segments, samples and results are those of
 * the plain octree walk (Sec. 4.2, "Rendering": the exact voxel crossings).
 * Reads the child array back to the host on `stream` (waiting for the
 * stream), checks it as po_tree_validate does, and allocates the index on
 * the current device (n_top * 32 + n_bricks * 2048 bytes, a few percent of
 * the leaf records); the handle owns it until po_tree_destroy.  Trees of
 * depth < 4 need none (PO_OK, nothing built); a second call is a no-op.  Must
 * not run while work that uses the handle is queued or running.  Errors:
 * PO_ERR_INVALID (NULL), PO_ERR_TREE (malformed child array: the handle is
 * unchanged and renders walk the caller's array, counting malformed entries
 * as device errors), PO_ERR_UNSUPPORTED (2^29 - 2 leaves or more, or an
 * index of 4 GiB or more), PO_ERR_OOM, PO_ERR_DEVICE. */
po_status po_tree_build_index(po_tree* t, void* stream);
/* po_tree_index_host: host only.  The traversal index po_tree_build_index
 * builds, from a host copy of a child array of depth D >= 4: writes *n_top
 * (nodes above level D - 3) and *n_bricks, and, when h_index is not NULL,
 * h_index[n_top * 8 + n_bricks * 512]: the renumbered nodes' child entries
 * (an entry >= n_top names brick entry - n_top), then the bricks, entry
 * slot1 * 64 + slot2 * 8 + slot3 of a brick (the child slots of the three
 * levels below its cube) being ((leaf + 1) << 2) | (D - level) of the leaf
 * holding that finest cell, 0 << 2 for empty space.  Call with NULL first
 * for the sizes.  Errors: as po_tree_validate, PO_ERR_INVALID (depth < 4),
 * PO_ERR_UNSUPPORTED (as po_tree_build_index). */
po_status po_tree_index_host(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child, int64_t n_leaves,
                             int64_t* n_top, int64_t* n_bricks, int32_t* h_index);
/* po_tree_destroy: releases the handle; if it holds a traversal index, waits
 * for the index's device to finish its work and frees it. */
po_status po_tree_destroy(po_tree* t);

/* ------------------------------------------------------------------ render
 * po_render_rays: renders n rays into d_rgb[n][3]; with PO_OUT_AUX also
 * d_aux[n][4].  The colour is sum_i T_i (1 - exp(-sigma_i delta_i)) c_i +
 * T_N bg over the data segments met before the early stop (Sec. 3 eqn:quad,
 * App. B.3), c_i = sigmoid(sum_k sh[leaf][ch][k] Y_k(d)) (Sec. 4.1).
 * Lists of at least 65536 rays are rendered in pieces as po_render_camera
 * describes (same queue, same equality up to rounding; with PO_OUT_AUX the
 * sample and cell counts are summed over the pieces, a cell cut between two
 * pieces counted once).
 * Errors: PO_ERR_INVALID (NULL tree/opts/arrays with n > 0, n < 0, bad
 * options), PO_ERR_DEVICE (launch failure). */
po_status po_render_rays(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                         const po_render_opts* opts, float* d_rgb, float* d_aux, void* stream);

/* po_render_camera: renders a camera image into d_rgb[height][width][3]
 * (and d_aux[height][width][4] with PO_OUT_AUX).  width, height in
 * [1, 16384]; fx, fy non-zero.
 * Images of at least 65536 pixels are rendered in pieces: every ray is walked for a bounded number of cells, the rays with
 * cells left are cut into parameter intervals walked in parallel, and the
 * pieces are composited front to back (compositing is associative, Sec. 3
 * eqn:quad), the piece holding the early stop walked again with the known
 * transmittance.  The colour equals the one-pass render (po_render_batch)
 * up to float rounding; where T lands within rounding of stop_T the two can
 * stop one cell apart, which moves at most stop_T of weight.  For this the
 * library keeps a work queue of about 200 MB per (device, stream), made on
 * the first such call and held until the process ends (if it cannot be
 * allocated, the image is rendered in one pass).  Calls on one stream are
 * ordered; calls on different streams use different queues.  Errors as for
 * po_render_rays. */
po_status po_render_camera(const po_tree* t, const po_camera* cam, const po_render_opts* opts,
                           float* d_rgb, float* d_aux, void* stream);

/* po_render_camera_noalloc: po_render_camera for callers that cannot
 * allocate device memory -- code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  It takes the same arguments,
 * writes the same outputs and returns the same errors, but calls no
 * hipMalloc, hipFree or allocating library routine: its work queue is a
 * fixed array of 100,663,808 bytes that the library holds in a static
 * device variable, one copy on each GPU it runs on, kept until the
 * process ends.  Its device address is looked up on the first call on a
 * device.  The queue holds 64 regions of 8192 pieces (half of the
 * per-stream queue); a long walk that finds its region full is finished by
 * its own lane, which changes the speed, not the result beyond float
 * rounding.  Images of more than 2^22 pixels (4,194,304; e.g. 2048 x 2048)
 * are rejected with PO_ERR_INVALID before any work is queued: render those
 * with po_render_camera.
 * Every call on one GPU shares that GPU's array, whatever the stream, and
 * the array keeps the last call's contents (each call clears the counters
 * it needs): calls that overlap on one GPU race, so the caller orders them
 * (one stream, or events).  Calls on different GPUs are independent. */
po_status po_render_camera_noalloc(const po_tree* t, const po_camera* cam, const po_render_opts* opts,
                                   float* d_rgb, float* d_aux, void* stream);

/* po_camera_rays: writes the pixel-centre rays of a camera, in row-major
 * pixel order, as d_origins[H*W][3] (the camera position) and
 * d_dirs[H*W][3] (unit directions, evaluated in FP64 and rounded to float32).
 * Rendering these rays with po_render_rays gives the camera image up to the
 * float32 rounding of the directions.  Used to build ray batches for the
 * optimisation of Sec. 4.3.  Errors: PO_ERR_INVALID, PO_ERR_DEVICE. */
po_status po_camera_rays(const po_camera* cam, float* d_origins, float* d_dirs, void* stream);

/* -------------------------------------------------------------- gradients
 * Accumulates (+=) into d_grad_sigma[n_leaves] and d_grad_sh[n_leaves][sh_stride]
 * the gradient of L with respect to the raw leaf values, given
 * d_grad_rgb = dL/dC [n][3] and the colours d_rgb_fwd [n][3] that
 * po_render_rays produced for the same rays and options (App. B.3: the first
 * pass stores the full colour, this second pass walks the same segments and
 * subtracts a running prefix; dC/dsigma_i = delta_i (c_i T_{i+1} - (C -
 * P_i)), zero where the raw density is <= 0; dC/dc_i = w_i, then the chain
 * rule through the sigmoid and the SH basis).  Several rays may hit one
 * leaf, so accumulation uses float atomics and its summation order is not
 * deterministic.  Zero the outputs first when a fresh gradient is wanted.
 * Batches of at least 65536 rays are differentiated in pieces: the rays
 * walked for a bounded number of cells are handed on as pieces whose
 * transmittance and colour prefix in front come from a forward pass over the
 * pieces, then every piece before the early stop is differentiated in
 * parallel (a cell cut between two pieces is two segments whose gradients add
 * up to the cell's).  Uses the work queue of po_render_camera.  The pieces
 * are cut as po_render_rays cuts the same n rays (and both run in one pass
 * below 65536 rays or with PO_ONE_PASS), so the transmittance in front of
 * every sample is the same float product in the render and here and the
 * backward stops on the sample where that render stopped: d_rgb_fwd must
 * come from a po_render_rays call with the same n and options (else, where a
 * ray's T lands within float rounding of stop_T, the two may stop one sample
 * apart and that ray's gradient is of the other stop point's colour).
 * Errors: PO_ERR_INVALID, PO_ERR_UNSUPPORTED (tree not PO_F32, or viewer
 * options sh_off / clip set), PO_ERR_DEVICE. */
po_status po_render_rays_backward(const po_tree* t, int64_t n, const float* d_origins,
                                  const float* d_dirs, const po_render_opts* opts,
                                  const float* d_rgb_fwd, const float* d_grad_rgb,
                                  float* d_grad_sigma, float* d_grad_sh, void* stream);

/* po_render_rays_keep and po_render_rays_backward_kept: the render and the
 * gradient of one ray batch as the two passes of App. B.3, where the second
 * pass reuses the pieces of the first instead of walking them forward again.
 * po_render_rays_keep renders like po_render_rays (no aux outputs or viewer
 * options; float32 trees) and leaves its pieces, with their forward results,
 * in the stream's work queue; d_ray_slot [n] int32 (device, caller-owned,
 * overwritten) records which rays it handed on.  po_render_rays_backward_kept
 * then accumulates the same gradient as po_render_rays_backward with d_rgb_fwd
 * from that render, without the forward pass over the pieces.  The backward
 * must be called on the same stream with the same tree, n, ray arrays,
 * d_ray_slot and options, and no other split render, split backward or kept
 * render may run on that stream's queue in between (the library checks these
 * on the host and returns PO_ERR_INVALID otherwise; it cannot check that the
 * contents of the arrays are unchanged).  One backward consumes the kept
 * pieces.  Below 65536 rays, or with PO_ONE_PASS, both run in one pass.
 * Errors: PO_ERR_INVALID, PO_ERR_UNSUPPORTED (tree not PO_F32, aux, sh_off or
 * clip set), PO_ERR_DEVICE. */
po_status po_render_rays_keep(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                              const po_render_opts* opts, float* d_rgb, int32_t* d_ray_slot, void* stream);
po_status po_render_rays_backward_kept(const po_tree* t, int64_t n, const float* d_origins,
                                       const float* d_dirs, const po_render_opts* opts,
                                       const float* d_rgb_fwd, const float* d_grad_rgb,
                                       float* d_grad_sigma, float* d_grad_sh, const int32_t* d_ray_slot,
                                       void* stream);

/* ------------------------------------------------------------ optimisation
 * Direct optimisation of the leaf values (Sec. 4.3; App. B.5): the NeRF
 * loss of Sec. 3 (eqn:nerfloss), reduced here as a mean over the batch and
 * the colour channels, minimised by plain SGD with the tree structure fixed.
 *
 * po_mse_grad: for n rays, d_grad_rgb[i][c] = scale * 2 (rgb - target) and
 * d_sq_sum[0] += sum of (rgb - target)^2 (one float; the caller zeroes it;
 * float atomics, so the last bits of the sum depend on scheduling).  scale =
 * 1 / (3 n) gives the gradient of the mean.  Errors: PO_ERR_INVALID,
 * PO_ERR_DEVICE.
 * po_sgd_step: d_param[i] -= lr * d_grad[i] for i < n and, if zero_grad is
 * non-zero, d_grad[i] = 0 in the same pass.  Errors: PO_ERR_INVALID
 * (NULL arrays with n > 0, n < 0, non-finite lr), PO_ERR_DEVICE. */
po_status po_mse_grad(int64_t n, const float* d_rgb, const float* d_target, float scale, float* d_grad_rgb,
                      float* d_sq_sum, void* stream);
po_status po_sgd_step(int64_t n, float* d_param, float* d_grad, float lr, int32_t zero_grad, void* stream);
/* po_gather_rays: the rows of a training batch (Sec. 4.3: random rays of the
 * training images), for i < n: d_bo[i] = d_o[d_idx[i]], d_bd[i] =
 * d_d[d_idx[i]] and d_bt[i] = d_t[d_idx[i]] (rows of 3 floats; d_idx int64
 * device indices, each in [0, n_src)).  The indices are checked on the
 * device: an index outside [0, n_src) gathers zeros and is counted by
 * po_device_errors.  Errors: PO_ERR_INVALID (NULL arrays with n > 0, n < 0,
 * n_src < 1), PO_ERR_DEVICE. */
po_status po_gather_rays(int64_t n, const int64_t* d_idx, int64_t n_src, const float* d_o, const float* d_d,
                         const float* d_t, float* d_bo, float* d_bd, float* d_bt, void* stream);
/* po_draw_batch: a training batch drawn on the device (Sec. 4.3: random rays
 * of the training images, uniform with replacement), so that a step needs no
 * index array: row i < n is row j_i = floor(z_i * n_src / 2^64) of the
 * source arrays, gathered as po_gather_rays gathers, where z_i is element
 * first + i (counting from 0) of the SplitMix64 sequence of `seed` (Steele,
 * Lea and Flood, OOPSLA 2014: z = seed + (k + 1) * 0x9E3779B97F4A7C15, then
 * z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *=
 * 0x94D049BB133111EB, z ^= z >> 31).  Consecutive batches of one fit take
 * consecutive ranges of the sequence (first = step * n), so a fit resumes
 * from (seed, step).  If d_sq_sum is not NULL, d_sq_sum[0] is set to 0 (the
 * accumulator po_mse_grad adds the batch's squared errors to).  Errors:
 * PO_ERR_INVALID (n < 0 or n >= 2^31, n_src < 1, NULL arrays with n > 0),
 * PO_ERR_DEVICE. */
po_status po_draw_batch(int64_t n, uint64_t seed, uint64_t first, int64_t n_src, const float* d_o, const float* d_d,
                        const float* d_t, float* d_bo, float* d_bd, float* d_bt, float* d_sq_sum, void* stream);

/* ---------------------------------------------------------------- batches
 * One job renders the 16x16 tiles [tile_begin, tile_end) of one camera
 * image of one tree (tiles numbered row-major over ceil(W/16) x ceil(H/16)).
 * po_render_batch renders up to PO_BATCH_MAX_JOBS jobs, of any trees and
 * image sizes, all on `stream`.  Jobs of fewer than 256 tiles (65536 pixels)
 * are rendered with as few kernel launches as their (dtype, SH degree)
 * groups allow, each ray walked to its end in one pass by one lane; their
 * pixels equal po_render_camera's bit for bit for images under 65536
 * pixels.  A job of 256 tiles or more (without PO_ONE_PASS in its options)
 * is rendered in pieces on its own, as
 * po_render_camera renders a large image (using the same work queue of
 * `stream`), and its pixels equal po_render_camera's up to float rounding
 * (bit for bit unless a region of the work queue filled up in one of the
 * two).  Errors: as po_render_camera, plus PO_ERR_INVALID for n_jobs outside
 * [0, PO_BATCH_MAX_JOBS] or a tile range outside the image. */
typedef struct {
    const po_tree* tree;
    po_camera cam;
    po_render_opts opts;
    float* d_rgb;       /* [height][width][3] */
    float* d_aux;       /* [height][width][3] or NULL */
    int32_t tile_begin, tile_end;
} po_job;
po_status po_render_batch(int32_t n_jobs, const po_job* jobs, void* stream);
/* Number of 16x16 tiles of a camera image. */
po_status po_camera_tiles(const po_camera* cam, int32_t* n_tiles);

/* -------------------------------------------------------------- compression
 * po_codebook_build: host only.  The codebook compression of App. B.2:
 * for each basis function k the RGB coefficient triples (coefficient (c, k)
 * of h_coef[leaf][coef_stride], channel-major as in the SH records) of all
 * leaves are quantised by median cut into at most M <= 65536 colours.  The
 * cut is fixed exactly so that results are reproducible: repeatedly split the
 * box whose longest side is longest (ties: lowest box number) along that side
 * (ties: lowest axis), the lower half being the floor(m/2) points first in
 * the order (coordinate, leaf index) and keeping the box number, the upper
 * half taking the next number; boxes of one point or zero extent are not
 * split.  A box's colour is the mean of its points, summed in double
 * precision in leaf order and rounded to float16 (nearest, ties to even).
 * Writes h_codebook[K][M][4] float16 bits (r, g, b, 0; unused entries 0),
 * h_index[n_leaves][index_stride] uint16 (positions k >= K set to 0) and, if
 * h_boxes is not NULL, the number of boxes used per basis function.  Uses up
 * to 16 host threads; the result does not depend on their number.  Errors:
 * PO_ERR_INVALID (bad sizes, NULL arrays, non-finite coefficients),
 * PO_ERR_OOM. */
po_status po_codebook_build(int64_t n_leaves, int32_t K, const float* h_coef, int64_t coef_stride, int32_t M,
                            uint16_t* h_codebook, uint16_t* h_index, int64_t index_stride, int32_t* h_boxes);

/* --------------------------------------------------------------- filtering
 * The visibility filter of the conversion from a dense density grid (Sec.
 * 4.2, "Filtering"): alpha maps of the training views are rendered through
 * the tree, every leaf keeps the largest weight of a segment in it, and the
 * leaves whose weight stays below a threshold are removed before the octree
 * is rebuilt (po_tree_leaf_cells, then po_builder_* on the kept cells).
 *
 * po_leaf_weights renders one camera (pixel-centre rays as po_render_camera,
 * early stop and step cap from opts) and raises d_weight[n_leaves] in place
 * to the largest weight of every data segment met: PO_WEIGHT_ALPHA the
 * segment's 1 - exp(-sigma delta), as the paper states the weight;
 * PO_WEIGHT_CONTRIB its contribution T (1 - exp(-sigma delta)) to the pixel.
 * With either, the early stop leaves voxels hidden behind opaque ones at
 * their initial weight.  d_weight must hold non-negative, non-NaN floats
 * (zeros before the first camera); the maximum is taken with integer atomics
 * on the float bits, so it does not depend on the order of rays or cameras.
 * d_alpha (or NULL) receives the alpha map [height][width], 1 - T.  Only the
 * densities are read; bg is ignored, and opts must not set flags, sh_off or
 * a slicing plane.  Errors: PO_ERR_INVALID, PO_ERR_UNSUPPORTED (viewer
 * options), PO_ERR_DEVICE. */
#define PO_WEIGHT_ALPHA 0
#define PO_WEIGHT_CONTRIB 1
po_status po_leaf_weights(const po_tree* t, const po_camera* cam, const po_render_opts* opts, int32_t mode,
                          float* d_weight, float* d_alpha, void* stream);

/* po_tree_leaf_cells: host only.  Checks the child array as
 * po_tree_validate does and writes h_cells[n_leaves][4] = (level, i, j, k),
 * the cell of each leaf (coordinates in [0, 2^level), child slot 4x + 2y + z
 * as in the builder); leaves that no entry references get (-1, -1, -1, -1).
 * Errors: PO_ERR_INVALID, PO_ERR_TREE, PO_ERR_OOM. */
po_status po_tree_leaf_cells(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child, int64_t n_leaves,
                             int32_t* h_cells);

/* -------------------------------------------------------------- statistics
 * po_traversal_stats: walks every pixel-centre ray of a camera through the
 * tree once, as the one-pass render does (Sec. 4.2, "Rendering": the exact
 * segments between voxel boundaries, early stop on the transmittance), and
 * writes h_stats[4] = {rays, data samples, cells visited, child entries read}
 * summed over the image: a data sample is a segment of positive length in a
 * data leaf before the early stop (the samples column of the aux output),
 * cells are the steps of the walk, and child entries are the 4-byte node
 * reads of its descents (each descent restarts below the deepest ancestor
 * shared with the previous cell).  These are the per-frame unit counts of the
 * render's algorithmic bytes.  Only densities are gathered; bg and colours
 * play no part.  Synchronous: waits for `stream`; concurrent calls are
 * serialised.  opts must not set flags, sh_off or a slicing plane.  Errors:
 * PO_ERR_INVALID, PO_ERR_UNSUPPORTED (viewer options), PO_ERR_DEVICE. */
po_status po_traversal_stats(const po_tree* t, const po_camera* cam, const po_render_opts* opts, int64_t* h_stats,
                             void* stream);
/* po_traversal_stats_rays: the same for the n rays (d_origins, d_dirs) as
 * po_render_rays takes them, each walked to its end in one pass; n == 0
 * writes zeros. */
po_status po_traversal_stats_rays(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                                  const po_render_opts* opts, int64_t* h_stats, void* stream);

/* --------------------------------------------------------------- resources
 * po_reserve_queues: allocates now the work queue that split renders,
 * split ray lists and split backward passes on `stream` use (about 200 MB on
 * the current device, held until po_release_queues or the end of the
 * process), so that the first such call on the stream allocates nothing.
 * Does nothing if the queue exists.  Errors: PO_ERR_DEVICE (allocation
 * failed; later calls then render in one pass).
 * po_release_queues: frees the work queues of the split render (one per
 * device and stream that rendered in pieces; see po_render_camera) after
 * waiting for all work on each of their devices.  Later split renders make
 * new ones.  Call it from one thread while no render is being issued.
 * Errors: PO_ERR_DEVICE (a wait or free failed; the remaining queues are
 * still released). */
po_status po_reserve_queues(void* stream);
po_status po_release_queues(void);

/* ----------------------------------------------------------------- errors
 * Device error counter: malformed child entries met and traversal step caps
 * hit, summed over all kernels since load or the last reset.  Reading
 * synchronises the current device. */
po_status po_device_errors(int64_t* count);
po_status po_device_errors_reset(void);
const char* po_status_str(po_status s);
const char* po_last_error(void);
/* Library version string, e.g. "plenoctree-mi355x 0.1 gfx950". */
const char* po_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PLENOCTREE_H */
