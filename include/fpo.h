/*
 * fpo.h -- C ABI of libfpo, the MI355X (gfx950) Fourier PlenOctree render
 * and fine-tune library.
 *
 * Paper: Wang et al., "Fourier PlenOctrees for Dynamic Radiance Field
 * Rendering in Real-time", CVPR 2022.  The scene lives in the leaves of a
 * union octree (Sec. 4.2); each leaf stores the Fourier coefficients
 * k^sigma (n1 = 31) and k^z (n2 = 5 per SH coefficient, 9 SH coefficients
 * per RGB channel) of Eq. 6 (Sec. 4.1).  Rendering at time t inverts them
 * with the real IDFT of Eq. 7-9, evaluates the SH colour of Eq. 1 (Sec. 3)
 * and composites front to back; fine-tuning back-propagates the L2 loss of
 * Eq. 13 (Sec. 4.3) into the coefficients.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Scene: the unit cube [0,1]^3.  A leaf (d, i, j, k) covers
 *   [i, i+1) 2^-d x [j, j+1) 2^-d x [k, k+1) 2^-d, 1 <= d <= FPO_MAX_DEPTH.
 * - Leaf coefficient order (166 values): q < 31 is k^sigma_q; then
 *   q = 31 + (c * 9 + j) * 5 + i is k^z for RGB channel c, SH index
 *   j = l*l + l + m (real SH, Condon-Shortley phase) and Fourier index i.
 * - Density: sigma_eff = sigma_scale * max(sigma(t), 0) per unit length.
 * - Coefficient store ("leaf records"): each leaf slot owns one record of R
 *   16-byte words, R = 48 (FPO_F32), 24 (FPO_BF16) or 16 (FPO_FP8_E4M3), i.e.
 *   768, 384 or 256 bytes; word g of slot l sits at byte offset
 *   16 * (l * R + g) and packs coefficients q = W g ... W g + W - 1 with
 *   W = 4, 8 or 16 per word.  Slots past q = 165 hold zero.  Records start on
 *   128-byte boundaries, so the 31 density coefficients of a leaf share one
 *   cache line.  Quantised stores carry a per-leaf FP32 scale:
 *   value = scale[leaf] * code.
 * - Snapshot records (baked values of one time): 32 values per leaf slot,
 *   F32 (128 bytes) or BF16 (64 bytes): value 0 = sigma(t) before activation,
 *   value 1 + c*9 + j = z_{c,j}(t), values 28..31 zero.
 * - Leaves are numbered by Morton slot (the order fpo_build_tree assigns);
 *   leaf_stride >= n_leaves.
 * - Ownership: the caller owns every buffer.  The library allocates no
 *   device memory, creates no streams and keeps no global state except the
 *   thread-local error message and, for fpo_render_noalloc, a static scratch
 *   array on each device with its address cached per device.  Device work is enqueued on `stream` (a
 *   hipStream_t passed as void*, NULL = the null stream) and is
 *   asynchronous; kernel faults surface at the caller's next synchronisation.
 * - Errors: every call returns fpo_status.  On FPO_E_INVALID or
 *   FPO_E_UNSUPPORTED nothing is launched and outputs are untouched.
 *   FPO_E_DEVICE reports a HIP launch error.  fpo_last_error() returns a
 *   message for the last non-OK status on the calling thread.  Host calls
 *   that allocate host memory (fpo_build_tree, fpo_union_leaves,
 *   fpo_coarse_occupancy) return FPO_E_NOMEM when an allocation fails.
 * - Tracing: every call is a roctx range named after it (visible to
 *   rocprofv3 --marker-trace; free when no tool is attached).
 * - Debug switches (environment, read at each call):
 *   FPO_FAULT=alloc makes the host calls above fail their first allocation
 *   (FPO_E_NOMEM), to exercise callers' error paths;
 *   FPO_FORCE_FALLBACK=1 makes fpo_render and fpo_render_noalloc ignore the
 *   skip flags and walk every whole chord (plain traversal), which must give
 *   the image of the skip modes.
 */
#ifndef FPO_H
#define FPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FPO_OK = 0,
    FPO_E_INVALID = 1,      /* bad argument; nothing launched */
    FPO_E_UNSUPPORTED = 2,  /* valid but not compiled in (e.g. another layout) */
    FPO_E_DEVICE = 3,       /* HIP runtime error */
    FPO_E_CAPACITY = 4,     /* caller-provided capacity too small */
    FPO_E_NOMEM = 5         /* a host call could not allocate host memory */
} fpo_status;

typedef enum { FPO_F32 = 0, FPO_BF16 = 1, FPO_FP8_E4M3 = 2 } fpo_dtype;

#define FPO_N_SIGMA 31          /* n1 */
#define FPO_N_SH_FOURIER 5      /* n2 */
#define FPO_SH_DEGREE 2         /* l_max */
#define FPO_N_SH 9              /* (l_max + 1)^2 */
#define FPO_N_COEFF 166         /* n1 + 3 * 9 * n2 */
#define FPO_N_BAKED 28          /* sigma(t) + 27 SH coefficients */
#define FPO_BASIS_STRIDE 32     /* floats per row of a device basis table */
#define FPO_MAX_DEPTH 10

/* Learned proposal and coarse occupancy (not in the paper; see the proposal
 * section below). */
#define FPO_MLP_N_IN 7             /* entry point (3), unit direction (3), t / T mod 1 */
#define FPO_MLP_N_PE 84            /* 7 inputs x 6 frequencies x (sin, cos) */
#define FPO_MLP_HIDDEN 64
#define FPO_MLP_N_OUT 3            /* hit logit, s_in logit, s_out logit */
#define FPO_MLP_N_PARAMS 9795      /* [85][64] + [65][64] + [65][3], biases as last rows */
#define FPO_MLP_N_PARAMS_PADDED 9796
#define FPO_MLP_PACKED_BYTES 23056 /* FP16 matrix-core fragments + FP32 biases */
#define FPO_COARSE_RES 64
#define FPO_COARSE_WORDS 8192      /* 64^3 bits */
#define FPO_MAX_FRAMES 120         /* frames per fpo_dft_frames call (LDS: basis + staged records < 64 KB) */
#define FPO_PRUNE_SIGMA 1e-3f      /* Sec. 3: leaves below this density are dropped */
#define FPO_RENDER_SKIP_COARSE 1   /* fpo_render_opts.flags */
#define FPO_RENDER_SKIP_PROPOSAL 2
#define FPO_RAYS_RECORD 4          /* fpo_render_rays / fpo_render_backward: segment records */
#define FPO_RECORD_BYTES 32        /* one recorded segment in the workspace */

/* Fourier / SH sizes, period and density scale.  Only (31, 5, 2) is compiled. */
typedef struct {
    int32_t n_sigma;       /* n1 = 31 */
    int32_t n_sh_fourier;  /* n2 = 5 */
    int32_t sh_degree;     /* l_max = 2 */
    float period;          /* T of Eq. 8, in frames (60) */
    float sigma_scale;     /* s: density per unit length per unit ReLU(sigma) (64) */
} fpo_layout;

/* A built tree resident on the device. */
typedef struct {
    const int32_t* children;  /* device [n_nodes][8] int32: 0 empty, >0 node, <0 -(leaf slot + 1);
                                 node 0 is the root; octant = x | y << 1 | z << 2 */
    int64_t n_nodes;          /* 1 .. 2^26 - 1 (32-bit byte offsets into children) */
    int32_t max_depth;        /* 1 .. FPO_MAX_DEPTH */
    const void* coeffs;       /* device leaf records (see above) */
    const float* leaf_scale;  /* device [leaf_stride] for BF16 / FP8, ignored for F32 */
    fpo_dtype dtype;
    int64_t n_leaves;
    int64_t leaf_stride;
    fpo_layout layout;
    const int32_t* grandchildren; /* device [n_grandchild_rows][64][2] int32 from fpo_grandchild_tables
                                     of this view's children, or NULL.  Walks then descend two levels per
                                     read from the nodes it covers.  8-byte aligned. */
    int64_t n_grandchild_rows;    /* rows of grandchildren: nodes 0 .. n - 1 (1 .. min(n_nodes, 2^22 - 1));
                                     ignored when grandchildren is NULL */
    const int64_t* level_offsets; /* host [max_depth + 1], or NULL: the nodes of depth L are rows
                                     level_offsets[L] .. level_offsets[L + 1] - 1, as fpo_build_tree
                                     numbers them (0 first, n_nodes last, non-decreasing).  The
                                     pruning calls then clear empty subtrees one level per pass,
                                     bottom up, instead of passing over every row max_depth - 1
                                     times; with offsets that do not match the table the pruning
                                     may leave some empty subtrees in place (renders still equal) */
    const int32_t* bounds;        /* host [6] int32, or NULL (the unit cube): a box on the finest
                                     lattice (2^max_depth cells per axis) that holds every leaf,
                                     [bounds[0], bounds[3]) x [bounds[1], bounds[4]) x [bounds[2],
                                     bounds[5]), e.g. from fpo_leaf_bounds; 0 <= lo < hi <= 2^max_depth
                                     per axis.  fpo_render and fpo_render_noalloc without skip flags,
                                     fpo_render_rays, fpo_render_backward and fpo_trace_rays clip each
                                     ray to this box instead of the unit cube: a ray that misses it
                                     ends at once, the others start their walk on its face.  Outside
                                     the leaves there is nothing to composite (Eq. 2), so colours and
                                     gradients are the same up to FP32 rounding of the entry point; a
                                     box that cuts a leaf drops the part of it outside.  The skip
                                     modes, fpo_ray_labels and the fusion calls measure along the
                                     cube's chord and ignore it */
} fpo_tree_view;

/* Pinhole camera: ray through pixel centre (u + 0.5, v + 0.5), row 0 at the
 * top, y up.  right = normalise(fwd x up), up' = right x fwd;
 * direction = normalise(f + sx right + sy up') with
 * sx = (2 (u + 0.5) / W - 1) tan(fov_y / 2) W / H,
 * sy = (1 - 2 (v + 0.5) / H) tan(fov_y / 2). */
typedef struct {
    float eye[3], fwd[3], up[3];
    float fov_y_deg;
    int32_t width, height;
    double time;              /* t of Eq. 7-9, frames; any finite value (T-periodic) */
} fpo_camera;

#define FPO_CAMERA_FLOATS 16  /* floats per camera in a device camera table */

typedef struct {
    float bg[3];              /* background colour added with the final transmittance */
    float stop_T;             /* early termination: stop after the segment that drives
                                 T below stop_T; 0 disables */
    const void* snapshot;     /* NULL: Fourier mode.  Else device snapshot records
                                 [leaf_stride] (see above) of one time; the camera's time
                                 is unused */
    fpo_dtype snapshot_dtype; /* FPO_F32 or FPO_BF16 */
    int64_t snapshot_cam_stride; /* leaf records between consecutive cameras' (or time
                                    indices') snapshots; 0: all share one */
    int32_t flags;            /* 0: plain traversal.  fpo_render only:
                                 FPO_RENDER_SKIP_COARSE: each ray walks the octree only
                                 between the first and last set cells of coarse_bits on
                                 its chord;
                                 FPO_RENDER_SKIP_PROPOSAL: the proposal network predicts
                                 the first entry and last exit; the skipped prefix and
                                 suffix are checked against coarse_bits before the walk
                                 (where a check fails, the walk starts at the first or
                                 ends at the last set cell instead).
                                 Either way the image equals the plain render up to FP32
                                 rounding of the segment ends.
                                 fpo_render_rays and fpo_render_backward only:
                                 FPO_RAYS_RECORD: the forward (F32 Fourier mode, at most
                                 32768 rays) writes each ray's segments of positive optical
                                 depth into workspace; the backward of the same rays then
                                 treats them independently instead of re-walking the rays. */
    const uint32_t* coarse_bits; /* device [FPO_COARSE_WORDS] from fpo_coarse_occupancy of
                                    this tree (skip modes) */
    const void* proposal;     /* device FPO_MLP_PACKED_BYTES from fpo_mlp_pack
                                 (FPO_RENDER_SKIP_PROPOSAL) */
    void* workspace;          /* device scratch.  Skip modes: 8-byte aligned, at least
                                 min(n_cams, 16) * W * H * 8 bytes.  FPO_RAYS_RECORD:
                                 16-byte aligned; int32 [n_rays] counts (-1: the ray had more
                                 segments than fit), then from the next 256-byte boundary
                                 cap records of FPO_RECORD_BYTES per ray, ray-major, cap =
                                 (workspace_bytes - that offset) / (32 n_rays) >= 1; a record
                                 is {int32 leaf slot, delta, T before, colour before [3], 0, 0}.
                                 Written by fpo_render_rays, read by fpo_render_backward. */
    int64_t workspace_bytes;
} fpo_render_opts;

/* ---------------------------------------------------------------------- */
/* Host-side set-up                                                         */
/* ---------------------------------------------------------------------- */

/* Build the sparse union octree (Sec. 4.2: the union of the per-frame
 * structures; a leaf is a cell of the union) from its leaves.
 *   leaf_dijk    host [n_leaves][4] int32 (depth, i, j, k), caller order.
 *   children_out host [cap_nodes][8] int32, or NULL to query the node count.
 *   n_nodes_out  host, receives the number of internal nodes.
 *   perm_out     host [n_leaves] int64 or NULL: perm_out[slot] = caller index of
 *                the leaf stored at Morton slot `slot`.
 * Nodes are numbered breadth first (root 0); leaves in Morton (z-order) order.
 * FPO_E_INVALID: NULL leaf_dijk, n_leaves < 1, max_depth outside 1..10, a depth
 * outside 1..max_depth, a coordinate outside [0, 2^depth), duplicate leaves, or
 * a leaf inside another leaf.  FPO_E_CAPACITY: cap_nodes < node count (the
 * count is still written).  Runs on the calling thread; no device work. */
fpo_status fpo_build_tree(const int32_t* leaf_dijk, int64_t n_leaves, int32_t max_depth,
                          int32_t* children_out, int64_t cap_nodes, int64_t* n_nodes_out,
                          int64_t* perm_out);

/* The smallest box on the finest lattice (2^max_depth cells per axis) that
 * holds every leaf of the octree (Sec. 3: the leaves are the only cells with
 * content), for fpo_tree_view.bounds.
 *   leaf_dijk   host [n_leaves][4] int32 (depth, i, j, k), as for fpo_build_tree.
 *   bounds_out  host [6] int32: lo x, y, z, then hi x, y, z (half-open).
 * FPO_E_INVALID: NULL pointers, n_leaves < 1, max_depth outside 1..10, a depth
 * outside 1..max_depth or a coordinate outside [0, 2^depth).  Overlaps are
 * not checked (fpo_build_tree does).  Runs on the calling thread; no device work. */
fpo_status fpo_leaf_bounds(const int32_t* leaf_dijk, int64_t n_leaves, int32_t max_depth, int32_t* bounds_out);

/* Real Fourier basis of Eq. 8 evaluated in FP64 on the host and rounded to
 * FP32: basis_out[r * 32 + i] = IDFT_i(times[r]) for i < n_sigma, 0 for the
 * remaining slots.  basis_out: host [n_t][FPO_BASIS_STRIDE].  The result is
 * what the device calls below take as their basis table. */
fpo_status fpo_time_basis(const double* times, int32_t n_t, const fpo_layout* layout,
                          float* basis_out);

/* Pack cameras into rows of FPO_CAMERA_FLOATS floats (host) for
 * fpo_camera_rays: eye, unit forward, right * tan_x, up' * tan_y (FP32,
 * computed in FP64), width, height. */
fpo_status fpo_camera_pack(const fpo_camera* cams, int32_t n_cams, float* table_out);

/* ---------------------------------------------------------------------- */
/* Device calls                                                             */
/* ---------------------------------------------------------------------- */

/* Scatter caller-order coefficients into F32 leaf records.
 *   src    device [n_leaves][n1 + 27 n2] F32, caller order (166 per leaf for
 *          the default layout).
 *   perm   device [n_leaves] int64 from fpo_build_tree.
 *   layout NULL for (31, 5); else n1 in {11, 21, 31}, n2 in {5, 11} (Table 3's
 *          Fourier dimensions).  Records of other layouts hold
 *          ceil((n1 + 27 n2) / 4) words rounded up to a multiple of 8.
 *   dst    device [leaf_stride][R] 16-byte words (F32 records, R = 48 for the
 *          default layout); padding slots and slots >= n_leaves are written
 *          with zero.
 * Layouts other than (31, 5) are accepted by fpo_quantize, fpo_render
 * (Fourier mode from F32, BF16 and FP8 stores without skipping; snapshot
 * mode: any) and fpo_bake_times (every store and output) only; every other
 * call returns FPO_E_UNSUPPORTED for them. */
fpo_status fpo_pack_coeffs(const float* src, const int64_t* perm, int64_t n_leaves,
                           int64_t leaf_stride, const fpo_layout* layout, float* dst, void* stream);

/* Render n_cams pinhole views (Sec. 4.1: per pixel, traverse the octree,
 * invert the leaf's coefficients at the camera's time with Eq. 7-9, colour
 * with Eq. 1, composite front to back).
 *   cams    host [n_cams].
 *   rgb_out device [n_cams][H][W][3] F32 (all cameras must share W and H).
 *   T_out   device [n_cams][H][W] F32 final transmittance, or NULL. */
fpo_status fpo_render(const fpo_tree_view* tree, const fpo_camera* cams, int32_t n_cams,
                      const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fpo_render with
 * the skip modes' scratch taken from a static device array of
 * FPO_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * (until the process ends) instead of opts->workspace, which is ignored.
 * Cameras go out in launches of as many as the array holds (at most 16).
 * Allocates nothing.  Every call on one device shares that device's array:
 * calls that overlap on one device (several streams or threads) race and must
 * be serialised by the caller; each launch rewrites every pixel's scratch
 * before reading it, so nothing needs clearing between calls.
 * FPO_E_CAPACITY (nothing launched) if one camera's scratch, 8 W H bytes,
 * exceeds FPO_NOALLOC_SCRATCH_BYTES.  Without a skip flag it is fpo_render. */
#define FPO_NOALLOC_SCRATCH_BYTES (32ll << 20)
fpo_status fpo_render_noalloc(const fpo_tree_view* tree, const fpo_camera* cams, int32_t n_cams,
                              const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream);

/* Generate rays for (camera, row, column) triples.
 *   cam_table device [n_cams][FPO_CAMERA_FLOATS] from fpo_camera_pack.
 *   cam, py, px device [n] int32; must index valid cameras / pixels.
 *   o_out, d_out device [n][3] F32; d_out is unit length. */
fpo_status fpo_camera_rays(const float* cam_table, int32_t n_cams, const int32_t* cam,
                           const int32_t* py, const int32_t* px, int64_t n,
                           float* o_out, float* d_out, void* stream);

/* Render arbitrary rays (Sec. 4.1: the per-pixel render of fpo_render for
 * rays given directly, each at its own time, as the fine-tuning of Sec. 4.3
 * draws them from the training images); ray r uses basis row t_idx[r] of the
 * Eq. 8 table that fpo_time_basis fills on the host in FP64.  In Fourier mode
 * from an F32 store, batches of at most 32768 rays run one ray per wave (the
 * lanes share each leaf's coefficients), larger ones one ray per lane; the
 * two agree to FP32 rounding.
 *   o, d   device [n_rays][3] F32 (d is normalised by the kernel; |d| > 0).
 *   t_idx  device [n_rays] int32 in [0, n_t).
 *   basis  device [n_t][FPO_BASIS_STRIDE] F32 (fpo_time_basis).
 *   rgb_out device [n_rays][3]; T_out device [n_rays] or NULL. */
fpo_status fpo_render_rays(const fpo_tree_view* tree, const float* o, const float* d,
                           const int32_t* t_idx, const float* basis, int32_t n_t, int64_t n_rays,
                           const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream);

/* Test support: the ordered leaf segments each ray crosses (no early stop):
 * the traversal of the sparse union octree (Sec. 4.2) that every render
 * above performs, exposed so that its visited-leaf lists can be compared.
 *   leaf_ids device [n_rays][max_visits] int32 Morton slots.
 *   t01      device [n_rays][max_visits][2] F32 entry / exit distance along the
 *            unit direction from o.
 *   n_visits device [n_rays] int32, the full count (may exceed max_visits, in
 *            which case only the first max_visits are written). */
fpo_status fpo_trace_rays(const fpo_tree_view* tree, const float* o, const float* d, int64_t n_rays,
                          int32_t max_visits, int32_t* leaf_ids, float* t01, int32_t* n_visits,
                          void* stream);

/* ---------------------------------------------------------------------- */
/* Fine-tuning (Sec. 4.3)                                                   */
/* ---------------------------------------------------------------------- */

/* Gradient of a loss L w.r.t. the leaf coefficients, through the render of
 * fpo_render_rays (Sec. 4.3: the IDFT is differentiable, so the photometric
 * loss of Eq. 13 back-propagates into the Fourier coefficients).  Without
 * FPO_RAYS_RECORD each ray's walk and shading are recomputed by one wave.
 * With it (opts->workspace as the forward left it, for the same rays, tree
 * values and opts), 8 waves share each ray's recorded segments, one wave per
 * segment, and only rays whose records overflowed are walked again; the
 * gradient is the same up to the order of the atomic additions.
 *   o, d, t_idx, basis, n_t, n_rays, opts: as passed to fpo_render_rays
 *            (opts->snapshot must be NULL; the store must be FPO_F32).
 *   rgb_fwd  device [n_rays][3], the forward colours of these rays.
 *   grad_rgb device [n_rays][3], dL/d rgb.
 *   grad_coeffs device F32 leaf records shaped like the coefficient store
 *            ([leaf_stride][192] floats); gradients are ADDED (FP32 atomics, so
 *            the summation order, and the last bits, vary run to run).
 * The early-termination decision is taken as in the forward pass and treated
 * as constant; the ReLU derivative at sigma = 0 is 0. */
fpo_status fpo_render_backward(const fpo_tree_view* tree, const float* o, const float* d,
                               const int32_t* t_idx, const float* basis, int32_t n_t, int64_t n_rays,
                               const fpo_render_opts* opts, const float* rgb_fwd, const float* grad_rgb,
                               float* grad_coeffs, void* stream);

/* L2 photometric loss of Eq. 13 over a batch of rays, as a mean over rays of
 * the squared RGB error: loss[0] += sum_r sum_c (rgb - target)^2 / n_rays,
 * grad_rgb = 2 (rgb - target) / n_rays.
 *   rgb      device [n_rays][3]; images device [n_images][height][width][3];
 *   image_idx, py, px device [n_rays] int32 (clamped into range);
 *   grad_rgb device [n_rays][3]; loss device [1] (accumulated, caller zeroes). */
fpo_status fpo_l2_loss(const float* rgb, const float* images, int32_t n_images, int32_t width,
                       int32_t height, const int32_t* image_idx, const int32_t* py, const int32_t* px,
                       int64_t n_rays, float* grad_rgb, float* loss, void* stream);

/* One Adam step (Kingma and Ba 2015; the paper names no optimiser) over n
 * floats, n a multiple of 4, all four buffers 16-byte aligned:
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps);
 * then g = 0.  step counts from 1. */
fpo_status fpo_adam_step(float* params, float* grad, float* m, float* v, int64_t n, float lr,
                         float beta1, float beta2, float eps, int32_t step, void* stream);

/* The same step with its count in device memory, for callers that capture the
 * fine-tuning step in a HIP graph: state is device int32[4], 16-byte aligned,
 * {step, c1, c2, unused} (c1, c2 as FP32 bits), zeroed by the caller before
 * the first step.  Each call (or replay of a captured call) adds one to the
 * step and applies the update of fpo_adam_step with that step. */
fpo_status fpo_adam_step_dev(float* params, float* grad, float* m, float* v, int64_t n, float lr,
                             float beta1, float beta2, float eps, int32_t* state, void* stream);

/* Adam on touched records only (lazy Adam; a semantic change from the dense
 * step above): params, grad, m, v are n_records records of record_floats
 * floats (a multiple of 4, at most 256; 192 for the F32 coefficient store),
 * 16-byte aligned.  A record whose gradient is zero everywhere is left as it
 * is: its parameters do not move and its moments do not decay.  Every other
 * record gets the update of fpo_adam_step and its gradient is cleared.  The
 * bias corrections come from `step` (>= 1), or, if state is not NULL, from
 * the device step count of fpo_adam_step_dev (advanced by one per call). */
fpo_status fpo_adam_step_touched(float* params, float* grad, float* m, float* v, int64_t n_records,
                                 int32_t record_floats, float lr, float beta1, float beta2, float eps,
                                 int32_t step, int32_t* state, void* stream);

/* ---------------------------------------------------------------------- */
/* Precision and time bake                                                  */
/* ---------------------------------------------------------------------- */

/* Quantise an F32 coefficient store (the paper states no precision; this is
 * the storage reading of this library).  Per leaf: scale = max |k| over its
 * n1 + 27 n2 coefficients for FPO_BF16, max |k| / 448 for FPO_FP8_E4M3 (OCP
 * E4M3FN), 1 for an all-zero leaf; code = round-to-nearest-even(k / scale)
 * with the quotient formed in FP32 (IEEE division), FP8 saturating at +-448.
 *   coeffs    device F32 leaf records of the layout ([leaf_stride][48] words
 *             for (31, 5); see fpo_pack_coeffs).
 *   layout    host, or NULL for (31, 5); any compiled (n1, n2).
 *   q_out     device leaf records of `dtype` for the layout ([leaf_stride][24]
 *             or [16] words for (31, 5)); code slots past the coefficients
 *             and leaves >= n_leaves are zero.
 *   scale_out device [leaf_stride] F32 (1 for leaves >= n_leaves). */
fpo_status fpo_quantize(const float* coeffs, int64_t n_leaves, int64_t leaf_stride, const fpo_layout* layout,
                        fpo_dtype dtype, void* q_out, float* scale_out, void* stream);

/* Evaluate Eq. 7 and Eq. 9 at n_t times for every leaf (a time bake), with
 * matrix-core (MFMA) contractions [times x K] x [K x leaves] in FP32 from 4
 * times on, and FP32 FMAs per leaf below (a per-frame decode).
 *   basis   device [n_t][FPO_BASIS_STRIDE] F32 (fpo_time_basis).
 *   out     device [n_t][leaf_stride] snapshot records of out_dtype (F32 or
 *           BF16, RNE), multiplied by the leaf scale for quantised stores;
 *           slots >= n_leaves are not written.  Record t is a snapshot for
 *           fpo_render / fpo_render_rays with snapshot_cam_stride = leaf_stride.
 *   sigma_out  device [n_t][leaf_stride] F32, or NULL: value 0 (sigma(t)) of
 *           each record written, as FP32 (the BF16 value itself for BF16
 *           records): the 4-byte plane fpo_prune_at_sigma reads instead of
 *           a whole record line per leaf.  Slots >= n_leaves are not written. */
fpo_status fpo_bake_times(const fpo_tree_view* tree, const float* basis, int32_t n_t, fpo_dtype out_dtype,
                          void* out, float* sigma_out, void* stream);

/* ---------------------------------------------------------------------- */
/* Occupancy at one time                                                    */
/* ---------------------------------------------------------------------- */
/* The union octree (Sec. 4.2) keeps every cell occupied in some frame; at a
 * time t a leaf whose sigma(t) (Eq. 7) is <= 0 has sigma_eff = 0 and adds
 * nothing to the image.  These calls read sigma(t) from snapshot records
 * (fpo_bake_times output), or its density plane, so that they agree with
 * the snapshot render.
 * A leaf is opaque at t iff sigma_scale * max(sigma(t), 0) > 0. */

/* Per-time child tables: children_out[t] is tree->children with every child
 * slot whose subtree holds no opaque leaf at time t set empty (0).  Rendering
 * snapshot t through a tree view whose children point at children_out[t]
 * walks fewer slots; every segment with positive optical depth is the same,
 * so the image equals the unpruned one up to FP32 rounding of segment ends at
 * ties.
 *   snapshots      device [n_t] snapshot records of snapshot_dtype,
 *                  snapshot_stride leaf records apart (>= n_leaves if n_t > 1).
 *   children_out   device [n_t][n_nodes][8] int32, 16-byte aligned.
 * Launches max_depth kernels; no allocation. */
fpo_status fpo_prune_at(const fpo_tree_view* tree, const void* snapshots, fpo_dtype snapshot_dtype,
                        int64_t snapshot_stride, int32_t n_t, int32_t* children_out, void* stream);

/* Two-level child tables for the walks' descents: one 8-byte read per two
 * levels instead of one 4-byte read per level.  Any child table (the union
 * octree's or a per-time table of fpo_prune_at) may be expanded; a view that
 * carries the result (fpo_tree_view.grandchildren) walks exactly the slots of
 * its children table, so every result is the same.
 *   children  device [n_t][n_nodes][8] int32, 16-byte aligned.
 *   n_rows    nodes 0 .. n_rows - 1 expanded (1 .. min(n_nodes, 2^22 - 1)).
 *             Nodes are numbered breadth first, so the nodes that have an
 *             internal child come first; expanding just those is enough.
 *   out       device [n_t][n_rows][64][2] int32, 16-byte aligned:
 *             out[t][x][8a + b] = (c, g) with c = children[t][x][a] and g =
 *             children[t][c][b] if 0 < c < n_nodes, else 0.
 * One kernel; no allocation. */
fpo_status fpo_grandchild_tables(const int32_t* children, int64_t n_nodes, int32_t n_t, int64_t n_rows,
                                 int32_t* out, void* stream);

/* fpo_prune_at with sigma(t) read from a density plane (fpo_bake_times
 * sigma_out) instead of the records: the same tables, from 4 bytes per leaf
 * and time instead of a record line.
 *   sigma         device [n_t][sigma_stride] F32 (>= n_leaves if n_t > 1).
 *   children_out  as fpo_prune_at. */
fpo_status fpo_prune_at_sigma(const fpo_tree_view* tree, const float* sigma, int64_t sigma_stride, int32_t n_t,
                              int32_t* children_out, void* stream);

/* The coarse occupancy of fpo_coarse_occupancy (64^3 cells, dilated by one
 * cell) over the leaves that are opaque at the snapshot's time only: the skip
 * modes of fpo_render accept it as opts->coarse_bits for renders of that
 * snapshot.
 *   leaf_cells device [n_leaves][4] int32 (depth, i, j, k) in slot order
 *              (the union leaves permuted by fpo_build_tree's perm), 16-byte
 *              aligned.
 *   snapshot   device snapshot records of one time.
 *   bits_out   device [FPO_COARSE_WORDS] uint32, overwritten. */
fpo_status fpo_coarse_occupancy_at(const int32_t* leaf_cells, int64_t n_leaves, int32_t max_depth,
                                   const void* snapshot, fpo_dtype snapshot_dtype, float sigma_scale,
                                   uint32_t* bits_out, void* stream);

/* ---------------------------------------------------------------------- */
/* Building a Fourier PlenOctree from per-frame PlenOctrees (Sec. 4.2)      */
/* ---------------------------------------------------------------------- */
/* Frames t = 0 .. T-1 sit at times t of Eq. 8 with period T (the basis is
 * T-periodic, so this is the paper's t = 1 .. T).  Per-frame values travel
 * as snapshot records (see above): 32 F32 values per leaf, value 0 = sigma,
 * 1 + c*9 + j = z_{c,j}, 28..31 zero.  Every tree involved (frames and
 * union) is built with the same max_depth. */

/* Leaves of the union of per-frame octree structures (Sec. 4.2: the union
 * has equal or deeper leaves than every frame).  A cell is a union leaf if no
 * given cell lies strictly inside it, some given cell covers it (itself or an
 * ancestor), and its parent is split.  Host call.
 *   leaf_dijk host [n_cells][4] (depth, i, j, k): the leaves of all frames,
 *             concatenated (duplicates allowed).
 *   union_out host [cap][4], Morton order, or NULL to query the count.
 * FPO_E_INVALID as for fpo_build_tree's range checks; FPO_E_CAPACITY if
 * cap < count (the count is still written). */
fpo_status fpo_union_leaves(const int32_t* leaf_dijk, int64_t n_cells, int32_t max_depth,
                            int32_t* union_out, int64_t cap, int64_t* n_union_out);

/* One frame's values on the union leaves (Sec. 4.2: a leaf divided in the
 * union copies the value of the frame leaf it lies in; a union leaf the
 * frame leaves empty gets zeros).
 *   frame_tree   the frame's own tree (fpo_build_tree of its leaves); only
 *                children, n_nodes, max_depth and n_leaves are read.
 *   frame_perm   device [frame leaves] int64, the perm of that build.
 *   frame_values device [frame leaves][32] F32 snapshot records, caller order.
 *   union_cells  device [n_union][4] int32 (depth, i, j, k) of the union
 *                leaves in the union tree's slot order.
 *   out          device [n_union][32] F32 snapshot records.
 *   n_bad        device [1] int32, incremented for every union cell that does
 *                not refine the frame (the frame is split below it); such
 *                cells get zeros. */
fpo_status fpo_frame_values(const fpo_tree_view* frame_tree, const int64_t* frame_perm,
                            const float* frame_values, const int32_t* union_cells, int64_t n_union,
                            float* out, int32_t* n_bad, void* stream);

/* Per-leaf DFT of Eq. 10-12: k_i = c_i sum_{t<T} x(t) IDFT_i(t) for the
 * density (i < 31) and every SH coefficient (i < 5), with c_0 = 1/T and
 * c_i = 2/T for i >= 1 (the least-squares projection onto Eq. 8, exact for
 * band-limited values), or the printed c_i = 1/T for every i if literal.
 *   frames      device [n_frames][leaf_stride][32] F32 snapshot records,
 *               16-byte aligned; 1 <= n_frames <= FPO_MAX_FRAMES.
 *   coeffs_out  device F32 leaf records ([leaf_stride][48] words), slots
 *               < n_leaves written (padding zero).
 *   sigma_max_out device [leaf_stride] F32 max_t sigma(t), or NULL (for
 *               pruning). */
fpo_status fpo_dft_frames(const float* frames, int32_t n_frames, int64_t n_leaves, int64_t leaf_stride,
                          int32_t literal, float* coeffs_out, float* sigma_max_out, void* stream);

/* Leaves to keep after fusion (Sec. 3: leaves with sigma < 1e-3 are
 * filtered out): indices l with sigma_max[l] >= threshold, ascending.  Host.
 *   keep_out host [n_leaves] int64; n_keep_out receives the count. */
fpo_status fpo_prune_leaves(const float* sigma_max, int64_t n_leaves, float threshold, int64_t* keep_out,
                            int64_t* n_keep_out);

/* ---------------------------------------------------------------------- */
/* PlenOctree fusion (Sec. 3, fine stage: Eq. 3-5)                         */
/* ---------------------------------------------------------------------- */
#define FPO_FIELD_MAX_GAUSS 8
#define FPO_FUSION_ACC 32          /* accumulator floats per leaf slot */

/* Analytic radiance field standing in for the generalizable network the
 * fusion queries (the network itself is not part of this library):
 *   sigma(x)  = sum_{g < n_gauss} a_g exp(-|x - mu_g|^2 / (2 w_g^2))   (stored units)
 *   c_c(x, d) = 1 / (1 + exp(-(u_c . x + v_c . d + b_c))),  c < 3, d unit. */
typedef struct {
    float mu[FPO_FIELD_MAX_GAUSS][3];
    float w[FPO_FIELD_MAX_GAUSS];
    float a[FPO_FIELD_MAX_GAUSS];
    int32_t n_gauss;
    float u[3][3];
    float v[3][3];
    float b[3];
} fpo_field;

/* Observe pass of one fusion view (Sec. 3: render a view of the PlenOctree
 * and query the points met with transmittance T > 1e-3).  Every pixel ray of
 * cam walks the static PlenOctree front to back with the transmittance of
 * the current values (sigma_eff = tree->layout.sigma_scale * max(sigma, 0)).
 * Each leaf segment [t0, t1) entered with T > tau is an observation at its
 * midpoint x along the ray direction d, weighted by its length delta:
 *   acc[l][0] += T delta           acc[l][1] += T delta sigma(x)
 *   acc[l][2 + 9c + j] += T delta Y_j(d) c_c(x, d)      acc[l][29] += delta
 * (Y the real SH of degree 2); the walk stops at the first segment entered
 * with T <= tau.  Only the tree structure of `tree` is used.
 *   values  device [leaf_stride][32] F32 leaf records in slot order: 0 = sigma,
 *           1 + 9c + j = z_{c,j} (the layout fpo_bake_times writes).
 *   acc     device [leaf_stride][FPO_FUSION_ACC] F32, ADDED to (FP32 atomics:
 *           the order of the sums is not fixed).  fpo_fusion_apply clears it. */
fpo_status fpo_fusion_observe(const fpo_tree_view* tree, const float* values, const fpo_camera* cam,
                              const fpo_field* field, float tau, float* acc, void* stream);

/* Apply pass: Eq. 3-5 once for every leaf observed in the view (acc[l][29]
 * > 0), with the view's length-weighted mean transmittance T_i = acc0 / acc29:
 *   sigma <- (W sigma + acc1 / acc29) / (W + T_i)
 *   z     <- (W z + acc[2 + q] / acc29) / (W + T_i)
 *   C <- C + 1;  W <- (C - 1) / C W + T_i / C
 * then clears acc[l].  Leaves not observed are left as they are.
 *   values device [n_leaves][32] F32 (as above), weight device [n_leaves] F32,
 *   count device [n_leaves] int32, acc device [n_leaves][FPO_FUSION_ACC]. */
fpo_status fpo_fusion_apply(float* values, float* weight, int32_t* count, float* acc, int64_t n_leaves,
                            void* stream);

/* ---------------------------------------------------------------------- */
/* Learned proposal (not in the paper)                                      */
/* ---------------------------------------------------------------------- */
/* A small MLP predicts, per ray and time, whether the ray meets a
 * contributing leaf and where the contributing part of its chord begins and
 * ends; rays use it to skip empty space (fpo_render_opts.flags).  Every skip
 * is checked against a dilated coarse occupancy grid, so the image does not
 * depend on how good the prediction is, only the speed.
 *
 * Network: inputs x = (entry point into the unit cube, unit direction,
 * t / T mod 1); positional encoding (sin 2^f pi x_c, cos 2^f pi x_c), f < 6,
 * feature 12 c + 2 f + {0 sin, 1 cos}; 84 -> 64 -> 64 -> 3, ReLU on the hidden
 * layers.  Parameters: FP32 [85][64], [65][64], [65][3] matrices laid end to
 * end (input index major, bias as the last row), FPO_MLP_N_PARAMS floats
 * (allocate FPO_MLP_N_PARAMS_PADDED for fpo_adam_step).  Training runs in
 * FP32; inference uses FP16 weights and activations with FP32 accumulation
 * on the matrix cores. */

/* Coarse occupancy of a tree: bit (z * 64 + y) * 64 + x of bits_out is set
 * iff a leaf overlaps coarse cell (x, y, z) of the 64^3 grid or one of its 26
 * neighbours.  Host call; arguments as for fpo_build_tree.
 *   bits_out host [FPO_COARSE_WORDS] uint32. */
fpo_status fpo_coarse_occupancy(const int32_t* leaf_dijk, int64_t n_leaves, int32_t max_depth,
                                uint32_t* bits_out);

/* Training labels from the plain walk at each ray's time, with the early
 * termination of opts->stop_T: hit = 1 if some segment has sigma_eff * delta
 * > 0 before the walk stops; s_in / s_out = entry of the first and exit of
 * the last such segment, as distances from the cube entry divided by the
 * chord length in the cube (0 when hit = 0).  Also writes the network inputs.
 *   o, d, t_idx, basis, n_t, n_rays: as for fpo_render_rays (Fourier mode).
 *   tau      device [n_t] F32, t / T mod 1 of each basis row.
 *   labels   device [n_rays][3] F32 (hit, s_in, s_out).
 *   inputs   device [n_rays][FPO_MLP_N_IN] F32; a ray that misses the cube
 *            gets its origin as entry point. */
fpo_status fpo_ray_labels(const fpo_tree_view* tree, const float* o, const float* d, const int32_t* t_idx,
                          const float* basis, const float* tau, int32_t n_t, int64_t n_rays,
                          const fpo_render_opts* opts, float* labels, float* inputs, void* stream);

/* FP32 forward pass (training precision).
 *   params device [FPO_MLP_N_PARAMS] F32; inputs device [n][7]; out device [n][3]. */
fpo_status fpo_mlp_forward(const float* params, const float* inputs, int64_t n, float* out, void* stream);

/* Floats of workspace fpo_mlp_loss_grad needs for a batch of n rays. */
int64_t fpo_mlp_workspace_floats(int64_t n);

/* Loss and gradient of a batch, in FP32.  Per ray: binary cross-entropy of
 * the hit logit against labels[.][0]; if labels[.][0] > 0.5, pinball losses
 * rho_q(y - sigmoid(o)) = (y - sigmoid(o)) (q - [y < sigmoid(o)]) with
 * q = 0.1 on s_in and q = 0.9 on s_out.  The batch loss is the mean over rays.
 *   inputs, labels device [N][7], [N][3]; idx device [n] int32 rows of the
 *            batch, or NULL for rows 0..n-1.
 *   workspace device, fpo_mlp_workspace_floats(n) floats, 16-byte aligned.
 *   grad     device [FPO_MLP_N_PARAMS] F32, gradients ADDED.
 *   loss     device [1] F32, batch loss ADDED.
 * Deterministic: fixed reduction order, no atomics. */
fpo_status fpo_mlp_loss_grad(const float* params, const float* inputs, const float* labels, const int32_t* idx,
                             int64_t n, float* workspace, float* grad, float* loss, void* stream);

/* Inference weights from the FP32 parameters: FP16 (round to nearest even)
 * matrix-core fragments and FP32 biases.
 *   packed_out device FPO_MLP_PACKED_BYTES, 16-byte aligned. */
fpo_status fpo_mlp_pack(const float* params, void* packed_out, void* stream);

/* Inference as used inside fpo_render (FP16 weights and activations, FP32
 * accumulation).  inputs device [n][7]; out device [n][3] logits. */
fpo_status fpo_mlp_infer(const void* packed, const float* inputs, int64_t n, float* out, void* stream);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char* fpo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FPO_H */
