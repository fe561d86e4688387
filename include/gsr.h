/*
 * gsr.h -- C ABI of the MI355X (gfx950) batched Gaussian-splatting RGB-D
 * sensor renderer.
 *
 * The renderer is the tile-based 3D Gaussian Splatting rasteriser that the
 * DISCOVERSE simulator (arXiv 2507.21981) uses as its engine's renderer
 * (Sec. III-A, "Renderer": sorting, splatting, spherical-harmonics colour and
 * alpha blending on the GPU) to produce its RGB and depth sensors (Sec. III-C:
 * alpha-compositing the colour and the camera-space z of the Gaussians), for
 * scenes made of a background node plus rigidly posed object and robot nodes
 * (Sec. III-B "Asset Formatting", Fig. 1), many environments and cameras at a
 * time (Sec. III-E, Throughput Report).
 *
 * Conventions (shared by every entry point):
 *  - All float data is IEEE FP32, C-contiguous, little endian.
 *  - Gaussian parameters are ACTIVATED values: scales > 0, opacities in
 *    [0, 1]; quaternions (w, x, y, z) need not be unit length (the renderer
 *    normalises them).  SH coefficients are [n][K][3] with K = (degree+1)^2,
 *    real SH with the Condon-Shortley phase, index l*l + (m + l); colour =
 *    max(0, sum_k sh_k Y_k(d) + 0.5) with d the unit vector from the camera
 *    centre to the Gaussian mean.
 *  - Cameras map world to camera coordinates with OpenCV axes (x right,
 *    y down, z forward); pixel (px, py) samples at (px + 0.5, py + 0.5).
 *  - A node pose maps node-local coordinates to world coordinates.
 *  - Outputs: rgb [n_envs][cams][H][W][3], depth [..][H][W] = sum of
 *    alpha*T*z (camera-space z of each Gaussian mean, unnormalised; 0 where
 *    nothing is hit), alpha [..][H][W] = 1 - final transmittance.
 *  - Every call returns a gsr_status code; nothing throws across the ABI.
 *    The message of the last failure is kept per context (gsr_last_error)
 *    or, for failures before a context exists, process-wide (ctx = NULL).
 *  - Calls taking a `stream` (a hipStream_t; NULL = the default stream) are
 *    asynchronous on it unless a flag says otherwise.  One context per host
 *    thread and stream; a context is not thread-safe.
 *  - Device-side failures (pair-capacity overflow, non-finite parameters)
 *    cannot be returned synchronously; they set the device status word read
 *    by gsr_query_status.  Non-finite Gaussians are culled and counted.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsr_context gsr_context; /* workspace, configuration, saved forward state, graphs */
typedef struct gsr_scene gsr_scene;     /* composed-scene metadata (node tables, block tables)   */

typedef enum {
    GSR_OK = 0,
    GSR_E_INVALID = -1,     /* bad argument (null pointer, negative size, unsupported value)  */
    GSR_E_NOMEM = -2,       /* device or host allocation failed                              */
    GSR_E_HIP = -3,         /* a HIP runtime call failed (no device, launch failure, ...)    */
    GSR_E_CAPACITY = -4,    /* pair capacity exceeded and automatic growth was not allowed   */
    GSR_E_UNSUPPORTED = -5, /* valid but not supported by this build (e.g. tile shape)       */
    GSR_E_STATE = -6        /* call order violated (e.g. backward with no saved forward)      */
} gsr_status;

/* One node's Gaussians in its node-local frame.  Device pointers, FP32. */
typedef struct {
    int64_t n;             /* number of Gaussians, >= 0                                  */
    int32_t sh_degree;     /* 0..3; all nodes of a scene share one degree                */
    int32_t reserved;
    const float* means;    /* [n][3]                                                     */
    const float* scales;   /* [n][3] activated (> 0)                                     */
    const float* quats;    /* [n][4] (w, x, y, z), any non-zero length                   */
    const float* opacities;/* [n]    activated, in [0, 1]                                */
    const float* sh;       /* [n][K][3]                                                  */
} gsr_gaussians;

/* Gradient buffers, same layout as gsr_gaussians (device pointers).  Each
   pointer may be NULL to skip that parameter. */
typedef struct {
    float* means;
    float* scales;
    float* quats;
    float* opacities;
    float* sh;
} gsr_gaussian_grads;

/* Rigid pose of a node, node-local -> world: x_world = R x_local + t.
   R row-major.  48 bytes. */
typedef struct {
    float R[9];
    float t[3];
} gsr_pose;

/* Pinhole camera.  80 bytes. */
typedef struct {
    float R[9];    /* world -> camera rotation, row-major                         */
    float t[3];    /* world -> camera translation: x_cam = R x_world + t          */
    float fx, fy;  /* focal lengths in pixels                                     */
    float cx, cy;  /* principal point in pixels                                   */
    float znear;   /* Gaussians with camera-space z <= znear are culled (> 0)     */
    float bg[3];   /* background colour composited behind the Gaussians           */
} gsr_camera;

/* Render flags. */
enum {
    GSR_FLAG_CHECK = 1u << 0,        /* synchronise the stream at the end of the call, read the
                                        status word, and on pair-capacity overflow grow the
                                        workspace and render again (at most twice).  Without it
                                        the call never synchronises; the caller checks
                                        gsr_query_status and re-renders on overflow.       */
    GSR_FLAG_SAVE = 1u << 1,         /* keep what gsr_render_backward needs (per-pixel final
                                        transmittance and contributor count, the sorted pairs and
                                        projected records).  Valid until the next render.    */
    GSR_FLAG_GRAPH = 1u << 2,        /* capture the launch sequence in a hipGraph on first use and
                                        replay it on later calls with the same arguments
                                        (pointers, sizes, flags); implies no synchronisation.
                                        Capacity must already suffice (overflow is reported). */
    GSR_FLAG_PERSISTENT = 1u << 3,   /* composite with a persistent grid walking a longest-list-
                                        first queue of (image, tile) work items                */
    GSR_FLAG_TIMING = 1u << 4,       /* record HIP events between the forward stages (eager
                                        calls only); read them with gsr_stage_times          */
    GSR_FLAG_AUGMENT = 1u << 5       /* apply the image-space augmentation bound by
                                        gsr_set_augment to rgb in the compositor's epilogue
                                        (not with GSR_FLAG_SAVE: the backward differentiates
                                        the plain image)                                     */
};

/* Status word contents (gsr_query_status). */
enum {
    GSR_STATUS_OVERFLOW = 1u << 0,   /* more tile-Gaussian pairs than the workspace holds     */
    GSR_STATUS_INTERNAL = 1u << 1    /* a tile list held an id outside its environment (a
                                        library defect; the entry was ignored)               */
};

typedef struct {
    uint32_t flags;          /* GSR_STATUS_* bits of the last render                          */
    uint32_t nonfinite;      /* Gaussians culled for non-finite parameters (summed over cams) */
    uint64_t pairs;          /* tile-Gaussian pairs the last render produced                  */
    uint64_t pair_capacity;  /* pairs the workspace holds now                                 */
    uint32_t max_tile_pairs; /* longest per-tile list of the last render                      */
    uint32_t reserved;
    uint64_t visible;        /* visible (image, Gaussian) projections                         */
    uint64_t visible_any;    /* Gaussians visible from at least one camera of their env       */
    uint64_t evals;          /* Gaussian-pixel evaluations of the last render: over pixels,
                                the list entries that reach the bounding box of the live
                                pixels of the pixel's wavefront sub-tile (taken per batch of
                                64 entries), evaluated up to and including the stopping one.
                                Counted only by renders with GSR_FLAG_CHECK (0 otherwise). */
} gsr_status_info;

/* Number of timed forward stages and their names, in order: views, project,
   gather (visible lists into per-image segments), depth_sort (the per-image radix
   sort by depth), chunks (each image's depth-ordered Gaussians cut into chunks of
   about equal pair counts), tile_counts (per chunk and tile), tile_ranges (per-tile
   slots and [start, end) ranges), emit, composite. */
#define GSR_STAGES 9

/* Configuration.  Tile shape must be one of 16x16, 16x8, 8x8, 32x8 (width x
   height).  Unset (zero) fields take defaults. */
typedef struct {
    int32_t tile_w, tile_h;   /* default 16 x 16                                             */
    int64_t pair_capacity;    /* initial pair capacity, default 1 << 22                       */
    int32_t persistent_grid;  /* persistent composite size in 256-thread blocks, default 8 per
                                 CU (scaled to the tile's block size)                        */
    int32_t pixels_per_thread;/* compositor pixels per thread, 1, 2 or 4 (default 2); capped
                                 at tile pixels / 64 (8x8 tiles use 1, 16x8 at most 2)       */
    int32_t stream_groups;    /* 1..4 (default 1): environments rendered as this many groups
                                 on the library's own streams, see gsr_render_rgbd           */
    int32_t reserved[5];
} gsr_config;

/* Per-image parameters of the image-space domain randomisation (Sec. IV-C,
   "Domain Randomization": random video overlays linearly blended into the
   stream, HSV-space augmentation, random gamma correction).  Applied per
   pixel in this order to the rendered colour x (background included):
     x = clamp(x, 0, 1); with an overlay frame o:
     x = (1 - overlay_weight) x + overlay_weight clamp(o, 0, 1);
     hexcone HSV of x (value = max channel, saturation = chroma / value, hue in
     turns): hue + hue_shift modulo 1, saturation * saturation_scale and
     value * value_scale each clamped to [0, 1], back to RGB;
     out = x ^ gamma per channel.
   32 bytes. */
typedef struct {
    float overlay_weight;    /* in [0, 1]; ignored without an overlay frame       */
    float hue_shift;         /* turns (1 = 360 degrees)                           */
    float saturation_scale;  /* >= 0                                              */
    float value_scale;       /* >= 0                                              */
    float gamma;             /* > 0                                               */
    float reserved[3];
} gsr_augment;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` (cfg may be NULL).  Allocates only
   small host state; workspace grows on first render.  Errors: GSR_E_HIP (no
   such device / runtime failure), GSR_E_UNSUPPORTED (tile shape),
   GSR_E_INVALID (out == NULL). */
int gsr_create(int device, const gsr_config* cfg, gsr_context** out);

/* Free the context and all its device workspace (synchronises the device).
   Scenes composed on it are detached: they can no longer be rendered, and
   gsr_scene_destroy still frees them. */
void gsr_destroy(gsr_context* ctx);

/* Message of the last failed call on ctx (ctx = NULL: process-wide last
   failure, e.g. from gsr_create).  Never NULL; owned by the library. */
const char* gsr_last_error(const gsr_context* ctx);

/* Current configuration, and a new tile shape or compositor pixels per thread
   (the next render uses them; cached graphs are dropped). */
int gsr_get_config(const gsr_context* ctx, gsr_config* out);
int gsr_set_tile(gsr_context* ctx, int32_t tile_w, int32_t tile_h);
int gsr_set_pixels_per_thread(gsr_context* ctx, int32_t ppt);

/* Stream groups (1..4) of later renders (gsr_render_rgbd).  With groups > 1 a
   render splits the scene's environments into that many contiguous groups of
   similar Gaussian counts (at most one group per environment).  Each group is
   rendered by a private sub-context with its own workspace on its own stream
   (default priority), forked from and joined back to the caller's stream, so
   one group's memory-bound stages (projection, sort) overlap another's
   compositing.  Every image is computed exactly as by a single-group render
   (same operations, same order per image).  Renders with GSR_FLAG_SAVE,
   GSR_FLAG_TIMING or GSR_FLAG_AUGMENT, and scenes of one environment, use one
   group.  After a grouped render gsr_query_status sums (ORs, maximises) the
   groups' counters, and gsr_copy_pairs, gsr_copy_pixel_state and
   gsr_stage_times return GSR_E_STATE.  More groups than the device's hardware
   queues less one (usually 3) serialise on shared queues.  Errors:
   GSR_E_INVALID (NULL ctx), GSR_E_UNSUPPORTED (groups outside 1..4). */
int gsr_set_stream_groups(gsr_context* ctx, int32_t groups);

/* ---- scene composition (Sec. III-B: background node + posed nodes) ----- */

/* Compose `n_envs` environments.  Environment e owns nodes
   [env_node_offsets[e], env_node_offsets[e+1]) of `nodes` (host array of
   n_nodes descriptors whose pointers are device memory); the first node of
   each environment is its background.  `poses` is a DEVICE array of n_nodes
   gsr_pose, read at every render (the caller updates it in place between
   simulation steps; background poses are normally identity).  The Gaussian
   data and the pose buffer are borrowed, not copied: they must stay valid
   while the scene is used.  Scene-global Gaussian ids follow the
   concatenation env-major, node order, local index.
   *inout: if non-NULL and the topology (env offsets, node sizes, SH degree)
   is unchanged, it is updated without allocating; otherwise a new scene is
   created (the old one is freed).  Synchronous.  Errors: GSR_E_INVALID
   (null pointers, n_envs < 1, bad offsets, n < 0, sh_degree outside 0..3 or
   differing between nodes, more than 2^31 - 1 Gaussians), GSR_E_NOMEM,
   GSR_E_HIP. */
int gsr_compose_scene(gsr_context* ctx, int32_t n_envs, const int32_t* env_node_offsets,
                      const gsr_gaussians* nodes, int32_t n_nodes, const gsr_pose* poses,
                      gsr_scene** inout);

/* Free a scene (NULL is a no-op), before or after its context. */
void gsr_scene_destroy(gsr_scene* scene);

/* Gaussian count of the scene, and of environment e. */
int64_t gsr_scene_gaussians(const gsr_scene* scene, int32_t env);

/* ---- rendering (Sec. III-A renderer, Sec. III-C RGB and depth sensors) --- */

/* Render every environment of `scene` from `cams_per_env` cameras each.
   cams: DEVICE array [n_envs * cams_per_env] of gsr_camera (env-major),
   read on the stream.  All images share width x height (1..8192).
   rgb (required), depth (required), alpha (nullable): DEVICE outputs laid
   out [n_envs][cams_per_env][height][width](x3 for rgb), fully written.
   flags: GSR_FLAG_*.  Stages, all on `stream`: node pose composition, EWA
   projection + SH colour + visible lists, per-image radix sort of the visible
   Gaussians by (depth bits, Gaussian id), per-tile pair counts and ranges,
   emission of the pairs into their tile buckets in that order, front-to-back
   compositing.
   Errors: GSR_E_INVALID (null ctx/scene/cams/rgb/depth, cams_per_env < 1,
   bad size), GSR_E_UNSUPPORTED (more than 13312 tiles per image or more than
   40000 tile-grid corners, more than 64 cameras per env), GSR_E_NOMEM,
   GSR_E_HIP, GSR_E_CAPACITY (with GSR_FLAG_CHECK, capacity still short after
   growing). */
int gsr_render_rgbd(gsr_context* ctx, const gsr_scene* scene, int32_t cams_per_env,
                    const gsr_camera* cams, int32_t width, int32_t height,
                    float* rgb, float* depth, float* alpha, uint32_t flags, void* stream);

/* Identifier of the render whose saved state gsr_render_backward would use:
   the last render, if it was made with GSR_FLAG_SAVE, else 0.  Also its image
   count (n_envs * cams_per_env) and size, so that a caller can check the shape
   of the upstream gradients it will pass.  Any output pointer but render_id
   may be NULL.  Host only, never blocks.  Errors: GSR_E_INVALID. */
int gsr_saved_render(const gsr_context* ctx, uint64_t* render_id, int32_t* images, int32_t* width,
                     int32_t* height);

/* Backward pass of the renderer: gradients of a scalar loss on the rgb, depth
   and alpha frames with respect to the Gaussians and the node poses.  The
   paper optimises Gaussian assets against image, depth and opacity terms
   (Sec. IV-B, mesh-to-Gaussian transfer and asset refinement) and places every
   node by a rigid pose (Sec. III-B); this call supplies both derivatives.
   render_id: the value gsr_saved_render gave right after the forward render
   (made with GSR_FLAG_SAVE on the same scene); if another render has replaced
   that state since, the call fails with GSR_E_STATE before any launch, so a
   backward can never pair its upstream gradients with another render's pairs.
   d_rgb [images][H][W][3] required; d_depth, d_alpha [images][H][W] nullable
   (zero upstream gradient); DEVICE buffers of exactly the saved render's shape
   (the library cannot check their size).
   grads: HOST array of n_nodes gsr_gaussian_grads (device pointers, node-local
   parameterisation: means, activated scales, unnormalised quaternions,
   activated opacities, SH), ACCUMULATED (+=), so the caller zeroes them.  The
   host array is read before the call returns and may be freed at once.
   d_poses: nullable DEVICE array [n_nodes][6], ACCUMULATED: per node
   (omega, rho), the derivative along the world-frame perturbation
   R' = exp([omega]x) R, t' = exp([omega]x) t + rho of its pose (R, t).
   Asynchronous on `stream` (no host synchronisation), so it can be captured
   in a graph; a captured backward stays valid while the context's workspace
   is not regrown (a later call with more images, Gaussians or nodes than any
   before it reallocates it).
   Errors: GSR_E_INVALID, GSR_E_STATE (no saved forward, or render_id is not
   it), GSR_E_NOMEM, GSR_E_HIP. */
int gsr_render_backward(gsr_context* ctx, const gsr_scene* scene, uint64_t render_id, const float* d_rgb,
                        const float* d_depth, const float* d_alpha, const gsr_gaussian_grads* grads,
                        float* d_poses, void* stream);

/* The same backward pass without any device allocation, for callers that
   cannot allocate (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, semantics and errors as
   gsr_render_backward, but its scratch (per-record gradients, 48 bytes per
   (image, Gaussian); the gradient-descriptor table; per-block pose sums) lives
   in a static device array of 256 MiB that each GPU the library runs on holds
   until the process ends, so the call never allocates.  Fails with
   GSR_E_CAPACITY (nothing launched) when the saved render needs more scratch
   than that (about 5.5 million (image, Gaussian) records).  Every call on one
   GPU shares that GPU's array: calls that overlap on one GPU (other streams,
   other contexts, other threads) race and give wrong gradients; calls on one
   stream are ordered and safe.  Needs the saved forward state, which the
   forward render allocated. */
int gsr_render_backward_noalloc(gsr_context* ctx, const gsr_scene* scene, uint64_t render_id,
                                const float* d_rgb, const float* d_depth, const float* d_alpha,
                                const gsr_gaussian_grads* grads, float* d_poses, void* stream);

/* ---- LiDAR by Gaussian ray tracing (Sec. III-C) ------------------------- */

/* One LiDAR ray: origin and unit direction in world coordinates; only
   Gaussians whose centre projects onto the ray at tmin < t < tmax count
   (tmin >= 0; a negative tmin is taken as 0).  32 bytes. */
typedef struct {
    float origin[3];
    float dir[3];
    float tmin, tmax;
} gsr_ray;

/* Build the acceleration structure the LiDAR tracer needs: one bounding-
   volume hierarchy per node over the node-local boxes of its Gaussians'
   ellipsoids at the Mahalanobis radius where each Gaussian's opacity can
   still give alpha >= 1/255 (3.33 sigma at opacity 1); poses are applied to
   the rays at trace time, so per-step pose updates need no rebuild.  Reads the Gaussian data back to
   the host; synchronous.  Call again after the Gaussian data changes or the
   scene is recomposed.  Errors: GSR_E_INVALID, GSR_E_NOMEM (also for more
   than 2^27 Gaussians or hierarchy nodes in a scene), GSR_E_HIP. */
int gsr_lidar_build(gsr_context* ctx, gsr_scene* scene);

/* Trace rays_per_env rays per environment (rays: DEVICE [n_envs *
   rays_per_env] gsr_ray, env-major) through the scene's Gaussians (Sec.
   III-C, LiDAR).  Per ray, a Gaussian's response is the peak of its density
   along the ray, alpha = min(0.99, opacity * exp(-D^2 / 2)) with D the
   smallest Mahalanobis distance from its centre to the ray; Gaussians with
   alpha >= 1/255 are composited front to back in the order of t = (mu - o) .
   d (ties by scene-global id) with the camera's stopping rule (before
   blending when T (1 - alpha) < 1e-4).  Outputs (DEVICE, [n_envs *
   rays_per_env]): range = sum alpha T t (unnormalised expected distance;
   divide by alpha), alpha = 1 - T, hits (nullable) = blended Gaussians.
   Asynchronous on `stream`.  Errors: GSR_E_INVALID (NULL arguments,
   rays_per_env < 1), GSR_E_STATE (gsr_lidar_build not called since the scene
   was composed), GSR_E_HIP. */
int gsr_render_lidar(gsr_context* ctx, const gsr_scene* scene, int32_t rays_per_env, const gsr_ray* rays,
                     float* range, float* alpha, uint32_t* hits, void* stream);

/* ---- mesh-to-Gaussian transfer (Sec. IV-B) ------------------------------ */

/* Convert a triangle mesh (a node's textured mesh, node-local frame) into
   Gaussians, one per facet (Sec. IV-B, "Mesh-Gaussian Transfer"): centre at
   the facet's barycentre; rotation whose columns are the unit edge a->b, n x
   t1 and the unit normal n = (b - a) x (c - a) / |..| (faces are (a, b, c));
   scales (d, d, flatten * d) with d the mean distance from the barycentre to
   the three vertices; opacity `opacity`; SH of degree sh_degree with the
   degree-0 coefficient (mean vertex colour - 0.5) * 2 sqrt(pi) (grey 0.5
   without vertex colours) and higher orders zero.  Degenerate facets (zero
   area) get opacity 0 and the identity rotation.
   vertices [n_vertices][3], vertex_colors [n_vertices][3] (nullable, in
   [0, 1]), faces [n_faces][3] int32: DEVICE inputs.  out: DEVICE arrays of
   n_faces Gaussians in the gsr_gaussians layout (means [n][3], scales [n][3],
   quats [n][4] unit (w, x, y, z), opacities [n], sh [n][K][3]), given through
   the non-const pointers of a gsr_gaussian_grads (NULL skips that array);
   the output can be composed directly as a node.  Synchronous on `stream`.
   Errors: GSR_E_INVALID (NULL arrays, negative sizes, sh_degree outside 0..3,
   flatten < 0, opacity outside [0, 1], or facets indexing outside the
   vertices -- those are written transparent and counted in the message),
   GSR_E_NOMEM, GSR_E_HIP. */
int gsr_mesh_to_gaussians(gsr_context* ctx, int64_t n_vertices, const float* vertices, const float* vertex_colors,
                          int64_t n_faces, const int32_t* faces, float flatten, float opacity, int32_t sh_degree,
                          const gsr_gaussian_grads* out, void* stream);

/* ---- image-space domain randomisation (Sec. IV-C) ----------------------- */

/* Augment `images` rendered frames: rgb [images][H][W][3] (DEVICE, read),
   overlay [images][H][W][3] (DEVICE, nullable: no overlay; the caller cuts and
   scales its video crops to the image size), params [images] gsr_augment
   (DEVICE), out [images][H][W][3] (DEVICE; may equal rgb).  Asynchronous on
   `stream`.  Errors: GSR_E_INVALID (NULL ctx, rgb, params or out; images < 1,
   width or height outside 1..8192), GSR_E_HIP. */
int gsr_augment_rgb(gsr_context* ctx, int32_t images, int32_t width, int32_t height, const float* rgb,
                    const float* overlay, const gsr_augment* params, float* out, void* stream);

/* Bind the augmentation that renders with GSR_FLAG_AUGMENT apply in the
   compositor's epilogue (the same arithmetic as gsr_augment_rgb on the
   rendered frame): params [images] (DEVICE, required), overlay
   [images][H][W][3] (DEVICE, nullable), both read at every such render, so
   the caller may redraw them in place between steps.  They must match the
   image count and size of those renders.  Host only.  Errors: GSR_E_INVALID. */
int gsr_set_augment(gsr_context* ctx, const gsr_augment* params, const float* overlay);

/* ---- status, inspection ------------------------------------------------ */

/* Synchronise the context's last stream and read the status word of the
   last render.  Errors: GSR_E_INVALID, GSR_E_HIP. */
int gsr_query_status(gsr_context* ctx, gsr_status_info* out);

/* Copy the sorted tile-Gaussian pairs of the last render (for tests and
   tools): keys[i] = (global tile << 32) | FP32 bit pattern of the
   camera-space z, values[i] = scene-global Gaussian id, ordered by (key,
   value); ranges[2*t], ranges[2*t+1] = [start, end) of global tile t, where
   global tile = image * tiles_per_image + ty * tiles_x + tx and image = env *
   cams_per_env + cam.  Device buffers: keys/values hold `capacity` entries,
   ranges 2 * total tiles.  *n_pairs receives the pair count.  Synchronous.
   Errors: GSR_E_INVALID, GSR_E_CAPACITY (capacity < pair count), GSR_E_STATE,
   GSR_E_HIP. */
int gsr_copy_pairs(gsr_context* ctx, uint64_t* keys, uint32_t* values, uint32_t* ranges,
                   int64_t capacity, int64_t* n_pairs);

/* Per-pixel saved forward state of the last render (device outputs, each
   [images][H][W]): final transmittance and the number of list entries up to
   and including the last blended one.  Either may be NULL.  Synchronous. */
int gsr_copy_pixel_state(gsr_context* ctx, float* T_final, uint32_t* n_contrib);

/* Per-stage durations (milliseconds, GSR_STAGES values) of the last render made
   with GSR_FLAG_TIMING.  Synchronises the context's last stream.  Errors:
   GSR_E_INVALID, GSR_E_STATE (no timed render), GSR_E_HIP. */
int gsr_stage_times(gsr_context* ctx, float* ms);

/* ---- autotuning -------------------------------------------------------- */

/* Time every supported tile shape, compositor pixels per thread and the
   persistent compositor on/off on this scene and camera set (full renders),
   keep the fastest in the context and return it (candidates are tried from
   16x16 tiles, one pixel per thread, one block per tile on; a later one
   replaces the choice only when at least 2% faster); then, for a scene of
   several environments, 1, 2 and 3 stream groups with that choice, timed as
   graph replays (the same 2% rule; gsr_get_config reports the groups kept).
   Outputs are scratch buffers sized for the call.  Synchronous.  The choice
   is cached per (images, width, height, Gaussian count) in the context. */
int gsr_autotune(gsr_context* ctx, const gsr_scene* scene, int32_t cams_per_env,
                 const gsr_camera* cams, int32_t width, int32_t height, float* rgb, float* depth,
                 float* alpha, int32_t* tile_w, int32_t* tile_h, int32_t* persistent, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
