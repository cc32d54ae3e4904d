/*
 * difftrans.h - C ABI of the MI355X recursive differentiable transparent-mesh
 * ray tracer (libdifftrans.so, HIP for gfx950).
 *
 * The method (paper Sec. 3.2-3.3): each camera ray is traced through a closed
 * triangle mesh of one transparent material.  At every surface hit it splits
 * into a reflected ray (Eq. 3) and a refracted ray (Snell, Eq. 4-6) blended
 * with the Fresnel weights R and T = 1 - R (Eq. 7-8); past the critical angle
 * only the reflected ray survives (total internal reflection); a segment
 * travelled inside the object is attenuated by exp(-sigma t) (Beer-Lambert,
 * Eq. 9-11, constant RGB absorption rate); a ray that leaves the object takes
 * the environment radiance of its direction.  The shading normal is the
 * barycentric blend of vertex normals (Eq. 12), normalised, each vertex normal
 * one third of the sum of the unit normals of the faces around the vertex
 * (Eq. 13, as written: not itself normalised).  The hit point is a
 * differentiable function of the three vertices of the first triangle hit, so
 * pixel losses back-propagate to vertex positions, the index of refraction and
 * the absorption rate (the interior derivative with the discrete path - which
 * triangles are hit, which splits are total internal reflections - held fixed).
 *
 * Conventions, for every call below:
 *  - All array pointers are DEVICE pointers owned by the caller, unless a
 *    comment says HOST.  The library never allocates device memory; every
 *    buffer it needs is sized by a *_bytes query and passed in by the caller.
 *  - Floating point arrays are float32, index arrays int32, row-major:
 *    V [nv][3], F [nf][3] (counter-clockwise seen from outside, so the
 *    geometric normal (v1-v0)x(v2-v0) points out), rgb [npix][3].
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Argument checks happen on the host before anything is queued;
 *    on a non-OK status nothing was queued.  Outputs are overwritten.
 *  - The IoR and sigma live in device memory so an optimiser can update them
 *    without a host synchronisation.
 *  - Errors are returned as dt_status; dt_last_error() gives a thread-local
 *    message for the last failing call on this thread.  No exceptions cross
 *    the ABI.  Data problems found on the device (a ray that leaves the object
 *    from inside, a shading normal on the wrong side, a full ray queue) are
 *    reported per pixel in the optional `flags` output and in `stats`.
 *  - The library keeps no global state besides that error string and the
 *    per-device build array of dt_build_bvh_noalloc.
 */
#ifndef DIFFTRANS_H
#define DIFFTRANS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dt_status;
#define DT_OK 0
#define DT_ERR_INVALID_ARGUMENT 1
#define DT_ERR_WORKSPACE_TOO_SMALL 2
#define DT_ERR_CAPACITY 3
#define DT_ERR_HIP 4
#define DT_ERR_UNSUPPORTED 5
#define DT_ERR_NOT_CONVERGED 6

/* per-pixel flags (bit set if any node of the pixel's ray tree had it) */
#define DT_FLAG_DEGEN 1     /* shading normal faced away; geometric normal used */
#define DT_FLAG_LEAK 2      /* a ray inside the object left it without a hit */
#define DT_FLAG_GRAZING 4   /* cos(theta_i) < 0.1 at some hit */
#define DT_FLAG_TIRB 8      /* |1 - sin^2(theta_t)| < 1e-2 at some hit */
#define DT_FLAG_TRUNC 16    /* some hit reached the depth cap */
#define DT_FLAG_OVERFLOW 32 /* a child ray was dropped: ray queue full */
#define DT_FLAG_STACK 64    /* BVH traversal stack overflowed (result invalid) */

#define DT_MAX_DEPTH 16
#define DT_STATS_LEN 64
/* stats layout (int64, device), written by dt_trace_forward:
 *   [g]      for g in 0..16: rays intersected in generation g
 *   [17 + g] for g in 0..16: of those, rays that hit the mesh
 *   [48] total rays, [49] dropped children, [50] generations run,
 *   [51] height of the BVH, [52] total hits */
#define DT_STAT_HITS 17
#define DT_STAT_TOTAL 48
#define DT_STAT_DROPPED 49
#define DT_STAT_GENERATIONS 50
#define DT_STAT_BVH_DEPTH 51
#define DT_STAT_TOTAL_HITS 52

/* ------------------------------------------------------------------ mesh */

/* Size of the caller-owned acceleration-structure blob and of the build
 * workspace for a mesh of nv vertices and nf faces (nv >= 3, 1 <= nf <= 2^26). */
dt_status dt_bvh_bytes(int32_t nv, int32_t nf, size_t* bvh_bytes, size_t* ws_bytes);

/* Build the scene acceleration data from V [nv][3] and F [nf][3]: unit face
 * normals, vertex normals (Eq. 13: one third of the sum of the unit normals of
 * the incident faces, in ascending face order, zero-area faces skipped), and a
 * linear BVH (63-bit Morton codes of face centroids, their top 32 bits up to
 * 2^20 faces, stable radix sort, binary
 * radix tree with index tie-break, bottom-up box fit, then small treelets
 * restructured for least box surface area, and a quantized 4-wide tree
 * collapsed from it for traversal).  Call again whenever V
 * changes.  Face indices must lie in [0, nv) (checked on the device only
 * through DT_FLAG results, not here: the caller guarantees it). */
dt_status dt_build_bvh(const float* V, int32_t nv, const int32_t* F, int32_t nf,
                       void* bvh, size_t bvh_bytes, void* ws, size_t ws_bytes, void* stream);

/* dt_build_bvh for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that must not call hipMalloc): the build
 * workspace is an array the library holds on each device (file-scope device
 * memory, DT_BVH_SCRATCH_BYTES per GPU, kept until the process ends) instead
 * of a caller-owned buffer.  Same outputs and conventions as dt_build_bvh; the
 * caller still owns V, F and the bvh blob.  Meshes whose build workspace
 * (dt_bvh_bytes' ws_bytes, about 65 bytes per face) exceeds
 * DT_BVH_SCRATCH_BYTES (about 500k faces) return DT_ERR_CAPACITY with nothing
 * queued.  No device memory is allocated, ever.  All calls on one GPU share
 * the one array, which keeps the last call's contents (the build clears what
 * it needs itself): two calls whose work overlaps on the same GPU (different
 * streams, or different host threads) race and corrupt each other's BVH, so
 * the caller must order them, e.g. on one stream. */
#define DT_BVH_SCRATCH_BYTES ((size_t)32 << 20)
dt_status dt_build_bvh_noalloc(const float* V, int32_t nv, const int32_t* F, int32_t nf,
                               void* bvh, size_t bvh_bytes, void* stream);

/* Copy the vertex normals held in a blob built for (nv, nf) to N [nv][3]. */
dt_status dt_bvh_vertex_normals(const void* bvh, int32_t nv, int32_t nf, float* N, void* stream);

/* ----------------------------------------------------------- environment */

#define DT_ENV_EQUIRECT 0
#define DT_ENV_MLP 1

/* Environment radiance as a function of direction (the environment is at
 * infinity).  EQUIRECT: texels [height][width][3], row 0 at the zenith (+y),
 * phi = atan2(x, -z), theta = polar angle from +y, u = phi/2pi + 1/2,
 * v = theta/pi, bilinear at texel coordinates (uW - 1/2, vH - 1/2), wrapping
 * in u, clamping in v.  MLP: input [d, sin(2^k pi d), cos(2^k pi d)] for
 * k < n_freq (at most 7), zero-padded to in_pad (64); n_layers (1-4) hidden
 * layers of width `hidden` (64 or 128) with ReLU; linear RGB head; bfloat16
 * weights ([out][in] row-major per layer, concatenated), float32 biases;
 * activations enter the bf16 matrix cores as three bf16 parts whose sum is
 * their float32 value, with float32 accumulation, so each layer is as accurate
 * as a float32 product.  Directions need not be unit: they are normalised
 * first.  Other shapes return DT_ERR_UNSUPPORTED.  d_texels (EQUIRECT only;
 * device [height][width][3], may be NULL): dt_trace_backward overwrites it
 * with dLoss/dtexel, from every ray that leaves the object (and, with
 * terminal_env, every ray stopped at the depth cap).  d_weights, d_biases
 * (MLP only; device float32 in the layout of weights and biases, both or
 * neither): dt_trace_backward overwrites them with dLoss/d(weights, biases)
 * of the network (the environment field's parameters, optimised with the
 * mesh, Sec. 3.1 "Environment Initialization" and Sec. 3.3 "Optimization"),
 * summed over every ray that leaves the object, with the ReLU pattern of
 * each lookup held fixed; supported for hidden width 64 (otherwise
 * DT_ERR_UNSUPPORTED, nothing queued).  Each entry is a sum of per-block
 * partial sums added in a fixed order, but which rays a block sums follows
 * the order of each generation's miss list, built with atomics, so the last
 * bits vary from run to run. */
typedef struct {
  int32_t kind;
  int32_t width, height;
  const float* texels;
  int32_t n_freq, n_layers, hidden, in_pad;
  const uint16_t* weights;
  const float* biases;
  float* d_texels;
  float* d_weights;
  float* d_biases;
} dt_env;

/* The environment seen by rays that leave the scene (the radiance a ray
 * gathers when it meets no surface, Sec. 3.3 "Recursive Ray Tracing"; the
 * environment is fitted before the object, Sec. 3.1 "Environment
 * Initialization").  rgb[i] = E(dirs[i]) for n directions (dirs, rgb:
 * device [n][3]). */
dt_status dt_env_query(const dt_env* env, const float* dirs, int64_t n, float* rgb,
                       void* stream);

/* grad_dirs[i] = (dE/dd)^T grad_rgb[i] (device [n][3] each). */
dt_status dt_env_query_backward(const dt_env* env, const float* dirs, int64_t n,
                                const float* grad_rgb, float* grad_dirs, void* stream);

/* ------------------------------------------------------------- tracing */

/* Spatially varying absorption rate mu_t(x) (Sec. 3.2: the radiance decay
 * along a ray inside the medium, Eq. 11 evaluated as a sum of the rate at
 * samples of the segment times their spacing).  An RGB grid of nx*ny*nz
 * nodes over the box [lo, hi]: node (i, j, k) sits at lo + (i/(nx-1),
 * j/(ny-1), k/(nz-1)) * (hi - lo) and holds mu[((k*ny + j)*nx + i)*3 + c].
 * mu_t(x) is the trilinear interpolant at x clamped into the box.  An
 * interior segment of length t from o along the unit direction d is
 * attenuated per channel by exp(-(t/S) sum_{s<S} mu_t(o + (s + 1/2)(t/S) d)),
 * the midpoint rule with S = samples steps.  With a grid the scene's sigma is
 * not used.  mu and d_mu are device arrays owned by the caller; d_mu (may be
 * NULL) receives dLoss/dmu from dt_trace_backward, which overwrites it.
 * Limits: 2 <= nx, ny, nz <= 1024, 1 <= samples <= 256, hi > lo per axis;
 * otherwise the calls that take the scene return DT_ERR_INVALID_ARGUMENT. */
typedef struct {
  const float* mu;     /* [nz][ny][nx][3] */
  int32_t nx, ny, nz;
  int32_t samples;
  float lo[3], hi[3];
  float* d_mu;         /* [nz][ny][nx][3] or NULL */
} dt_absorption;

/* Volumetric environment field outside the object: the exterior half of the
 * split of radiance into samples inside and outside the object (Sec. 3.3,
 * "Recursive Ray Tracing"), held as a coarse dense grid plus three planes
 * (the radiance-field representation of Sec. 3.1 "Environment
 * Initialization").  Inside the box [lo, hi] the feature of a point x
 * (4 channels) is the trilinear interpolant of the grid (node (i, j, k) at
 * lo + (i/(nx-1), j/(ny-1), k/(nz-1)) (hi - lo), value
 * grid[((k*ny + j)*nx + i)*4 + ch]) plus the bilinear interpolants of three
 * planes of res x res nodes, plane 0 over (x, y), 1 over (x, z), 2 over
 * (y, z), node (i, j) (i along the plane's first axis) at
 * planes[((p*res + j)*res + i)*4 + ch]; coordinates are clamped into the
 * box.  Channel 0 gives the density softplus(f0), channels 1-3 the colour.
 * Every exterior segment (camera ray to its first hit, a refracted or
 * reflected ray leaving the object to its next hit or to infinity) is clipped
 * to the box and sampled at the midpoints of S = samples equal steps h:
 * a_k = exp(-softplus(f0(x_k)) h), T_0 = 1, T_{k+1} = T_k a_k, emission
 * sum_k T_k (1 - a_k) c(x_k); the segment adds its emission and passes T_S
 * of the radiance beyond it.  Rays leaving the box see the environment map.
 * grid, planes: device float32 owned by the caller; d_grid, d_planes (both
 * or neither) receive dLoss/d(grid, planes) from dt_trace_backward, which
 * overwrites them (float atomics: the last bits vary from run to run).
 * Limits: 2 <= nx, ny, nz, res <= 1024, 1 <= samples <= 256, hi > lo per
 * axis, and the environment is an equirect map; otherwise the calls that
 * take the scene return DT_ERR_INVALID_ARGUMENT (DT_ERR_UNSUPPORTED for an
 * MLP environment). */
typedef struct {
  const float* grid;    /* [nz][ny][nx][4] */
  int32_t nx, ny, nz;
  const float* planes;  /* [3][res][res][4] */
  int32_t res;
  int32_t samples;
  float lo[3], hi[3];
  float* d_grid;        /* [nz][ny][nx][4] or NULL */
  float* d_planes;      /* [3][res][res][4] or NULL */
} dt_field;

typedef struct {
  const float* V;      /* [nv][3] */
  int32_t nv;
  const int32_t* F;    /* [nf][3] */
  int32_t nf;
  const void* bvh;     /* built by dt_build_bvh from this V, F */
  const float* ior;    /* [1]  IoR of the object, ambient medium 1 */
  const float* sigma;  /* [3]  RGB absorption per unit length */
  const dt_env* env;   /* HOST struct describing device data */
  const dt_absorption* absorb;  /* HOST struct or NULL: the constant rate sigma */
  const dt_field* field;        /* HOST struct or NULL: empty exterior */
} dt_scene;

/* Optional kernel timing (HOST struct of caller-created hipEvent_t handles):
 * when given, the forward records trace_events[2g] / [2g+1] around the
 * traversal kernel of generation g and mlp_events[2g] / [2g+1] around the
 * environment-MLP kernel of generation g (MLP environments only); the
 * backward records adjoint_events[2g] / [2g+1] around the adjoint kernel of
 * generation g and mlp_adjoint_events[2g] / [2g+1] around its MLP kernel.
 * Arrays must hold 2 * (max_depth + 1) events; NULL arrays are skipped. */
typedef struct {
  void* const* trace_events;
  void* const* adjoint_events;
  void* const* mlp_events;
  void* const* mlp_adjoint_events;
} dt_timing;

typedef struct {
  int32_t max_depth;          /* D in [0, 16]: generations 0..D are intersected,
                                 a hit in generation D is truncated */
  int32_t terminal_env;       /* 0: truncated hit contributes 0;
                                 1: it contributes A * E(d) */
  float t_eps;                /* minimum hit distance (1e-5) */
  int32_t checkpoint_stride;  /* backward: store every k-th generation and
                                 recompute the rest (1 = store all) */
  int64_t queue_capacity;     /* max rays per generation >= 1
                                 (0 = worst case n_rays * 2^g) */
  const dt_timing* timing;    /* optional, NULL = no event records */
} dt_trace_params;

/* Pinhole camera (HOST struct): right-handed, vertical FOV, image row 0 at
 * the top, one ray through each pixel centre.  Pixel (x, y) of this camera
 * is output pixel pixel_offset + y*width + x. */
typedef struct {
  float eye[3], target[3], up[3];
  float fov_deg;
  int32_t width, height;
  int64_t pixel_offset;
} dt_camera;

#define DT_RAYS_EXPLICIT 0
#define DT_RAYS_CAMERAS 1
typedef struct {
  int32_t kind;
  int64_t n;                 /* EXPLICIT: number of rays = pixels */
  const float* o;            /* EXPLICIT: origins [n][3] */
  const float* d;            /* EXPLICIT: unit directions [n][3] */
  int32_t n_cameras;         /* CAMERAS */
  const dt_camera* cameras;  /* CAMERAS: HOST array */
  int64_t n_pixels;          /* CAMERAS: size of the output pixel range */
} dt_rays;

/* Workspace and tape sizes for tracing n_rays camera rays against a mesh.
 * The tape carries the forward state the backward needs: every generation
 * when checkpoint_stride == 1, every k-th generation otherwise. */
dt_status dt_trace_bytes(const dt_trace_params* p, int64_t n_rays, int32_t nv, int32_t nf,
                         size_t* ws_bytes, size_t* tape_bytes);

/* Forward render: the recursive tracing procedure of Sec. 3.3 ("Recursive
 * Ray Tracing") over generations of rays - closest hit (Sec. 3.3
 * "Differentiable Mesh Intersection"), the shading normal of Eq. 12-13,
 * reflection and refraction directions (Eq. 3-6), Fresnel weights (Eq. 7-8),
 * total internal reflection, the attenuation of Eq. 11 on interior segments,
 * the environment at misses, the depth cap.  rgb [npix][3] (required), wtrunc [npix][3] (optional:
 * accumulated weight of truncated rays), flags [npix] (optional), path_sig
 * [npix] (optional: order-independent signature of each pixel's discrete
 * path, the sum mod 2^64 over its ray segments of SplitMix64's output
 * function applied to (g << 40) | (tir << 32) | (triangle + 1), with
 * triangle = -1 for a miss and tir = 0 for a truncated hit; two renders took
 * the same triangles and branches where the signatures agree), stats
 * [DT_STATS_LEN] int64 (optional).  tape may be NULL for a forward-only
 * render; when given it must be tape_bytes long and is later read by
 * dt_trace_backward with the same scene, rays and params. */
dt_status dt_trace_forward(const dt_scene* sc, const dt_rays* rays, const dt_trace_params* p,
                           float* rgb, float* wtrunc, int32_t* flags, uint64_t* path_sig,
                           int64_t* stats, void* tape, size_t tape_bytes, void* ws,
                           size_t ws_bytes, void* stream);

/* Backward: the reverse-mode derivative of the forward render (the
 * differentiable tracer of Sec. 3.3, "Differentiable Mesh Intersection" and
 * "Recursive Ray Tracing": through the hit distance and barycentrics, the
 * normals of Eq. 12-13, the directions of Eq. 3-6, the weights of Eq. 7-8 and
 * the attenuation of Eq. 11).  Given dLoss/drgb [npix][3], accumulate nothing and overwrite
 * dV [nv][3], d_ior [1], d_sigma [3] with dLoss/d(V, ior, sigma); with an
 * absorption grid, also its d_mu (when not NULL; d_sigma is then 0), and for
 * an equirect environment with d_texels set, dLoss/dtexel.  The gradients are
 * interior derivatives: the discrete path (triangles hit, TIR branches,
 * hit or miss, texel and grid cells) is held fixed.  Generations not stored on
 * the tape are recomputed from the nearest stored one.  dV and the grid and
 * texel gradients are sums whose order varies from run to run (float atomics,
 * or records ranked by an integer atomic), so their last bits do too; d_ior
 * and d_sigma are reduced in a fixed order. */
dt_status dt_trace_backward(const dt_scene* sc, const dt_rays* rays, const dt_trace_params* p,
                            const float* grad_rgb, const void* tape, size_t tape_bytes,
                            float* dV, float* d_ior, float* d_sigma, void* ws, size_t ws_bytes,
                            void* stream);

/* ------------------------------------------------- vertex reparameterisation */

/* The mesh optimiser's reparameterisation of the vertices, u = (I + lambda L) V
 * with L the combinatorial Laplacian D - A of the mesh's edge graph (the
 * preconditioned vertex update the appendix's training scheme takes from the
 * large-steps method it cites): solves (I + lambda L) x = b for the three
 * coordinate columns on the device, by Chebyshev iteration over the interval
 * [1, 1 + lambda m] that holds the matrix's eigenvalues (m: the largest
 * d_i + d_j over the edges, an upper bound of L's largest eigenvalue).  adj_off
 * [nv + 1], adj [adj_off[nv]]: each vertex's neighbours along edges (int32,
 * device, each undirected edge listed from both ends, no repeats).  b, x:
 * device float64 [nv][3]; x holds the starting guess on entry and the
 * solution on return.  Stops when every column's residual is within tol of
 * |b| (read back every 16 iterations: this call waits for the device, unlike
 * the others), or after max_iters iterations, returning DT_ERR_NOT_CONVERGED
 * then with x the last iterate.  iters_out, resid_out (HOST, may be NULL): the
 * iterations run and the largest relative residual.  The sums are reduced in
 * a fixed order, so the solve is bit-reproducible. */
dt_status dt_smooth_bytes(int32_t nv, size_t* ws_bytes);
dt_status dt_smooth_solve(const int32_t* adj_off, const int32_t* adj, int32_t nv, double lambda,
                          const double* b, double* x, double tol, int32_t max_iters,
                          int32_t* iters_out, double* resid_out, void* ws, size_t ws_bytes,
                          void* stream);

/* ---------------------------------------------------------- silhouette */

/* The silhouette (mask) term: each pixel's coverage by the object and the
 * gradient of a loss on it with respect to the vertices through the motion
 * of the object's outline - the visibility derivative the tracer's interior
 * derivatives do not carry (the paper's mask loss: Sec. 3.1 "Mask-based
 * Geometry Initialization"; the appendix on the ray tracer's mesh
 * regularization keeps it as a periodic term).
 *
 * The mask M_p of pixel p is the fraction of its unit square (pixel (x, y)
 * covers [x, x+1) x [y, y+1) in continuous image coordinates, row 0 at the
 * top) covered by the object's projection.  dt_mask_forward writes its value
 * at the pixel centre (1 where the centre's camera ray meets the mesh at
 * t > t_eps, else 0).  dt_mask_backward writes dLoss/dV for dLoss/dM given
 * per pixel: the boundary integral of the outline's normal velocity over the
 * outline inside each pixel, weighted by the pixel's dLoss/dM.  The outline
 * is made of silhouette edges (an edge whose two faces face opposite ways
 * as seen from the eye, or an edge with one face) at points whose camera
 * line meets no other triangle.  The integral is a fixed quadrature: an
 * edge whose projection is l pixels long gets n = max(1, ceil(rho l)) points
 * at the midpoints t_k = (k + 1/2)/n of its 3D parameter (from its lower to
 * its higher vertex index), weight |dx/dt| / n, each credited to the pixel
 * containing its projection; a point moves with its two vertices with
 * weights 1 - t_k and t_k.  The error against the exact integral falls like
 * 1/rho per pixel and 1/rho^2 summed over the image.
 *
 * rays: CAMERAS only, 1..DT_MASK_MAX_CAMERAS per call; mask, grad_mask:
 * device [n_pixels].  sc: V, F, nv, nf and bvh are used (env, ior, sigma and
 * absorb are not).  dV [nv][3] is overwritten (float atomic sums, order
 * varies run to run).  counts: device uint64 [3] or NULL: outline points in
 * an image whose pixel has a nonzero dLoss/dM, of those the visible ones,
 * and traversal stack overflows (such a point is treated as hidden).  ws:
 * dt_mask_bytes long (the edge list). */
#define DT_MASK_MAX_CAMERAS 16
dt_status dt_mask_bytes(int32_t nv, int32_t nf, size_t* ws_bytes);
dt_status dt_mask_forward(const dt_scene* sc, const dt_rays* rays, float t_eps, float* mask,
                          void* stream);
dt_status dt_mask_backward(const dt_scene* sc, const dt_rays* rays, const float* grad_mask, float rho,
                           float* dV, uint64_t* counts, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- serving */

/* A render server keeps several scenes resident and advances every admitted
 * request together: each dt_serve_step traces one surface interaction of every
 * live ray of every request (rays of requests admitted at different times,
 * with different scenes, environments, resolutions and depth caps share one
 * compacted queue), after first appending the camera rays of the requests
 * admitted in this call.  A request is finished when its slot has no live
 * rays left (slot_live[slot] == 0 after a step); its image is then complete in
 * the caller's pixel pool.  The ray/shading arithmetic is the tracer's, so a
 * request's image matches dt_trace_forward of the same camera up to the
 * order of the FP32 pixel additions. */
#define DT_SERVE_MAX_SCENES 8
#define DT_SERVE_MAX_ENVS 8
#define DT_SERVE_MAX_SLOTS 256

typedef struct {            /* one resident scene (device data, BVH built) */
  const float* V;
  int32_t nv;
  const int32_t* F;
  int32_t nf;
  const void* bvh;
  const float* ior;         /* [1] */
  const float* sigma;       /* [3] */
} dt_serve_scene;

typedef struct {            /* a request admitted by this step */
  int32_t slot;             /* request slot in [0, DT_SERVE_MAX_SLOTS), unused by live rays */
  int32_t scene;            /* index into scenes */
  int32_t env;              /* index into envs: the scene's own (render) or another (relight) */
  int32_t max_depth;        /* [0, 16] */
  dt_camera camera;         /* pixel_offset: first pixel of its image in the pool */
} dt_serve_admit;

/* Workspace of a server with queue_capacity live rays (both queues + scan). */
dt_status dt_serve_bytes(int64_t queue_capacity, size_t* ws_bytes);
/* Empty the queue (call once before the first step). */
dt_status dt_serve_reset(void* ws, size_t ws_bytes, int64_t queue_capacity, void* stream);
/* One step.  scenes, envs, admits: HOST arrays (equirect or MLP environments;
 * the misses lit by an MLP environment are listed and evaluated on the matrix
 * cores after the trace, one environment at a time); they reach the device as
 * a kernel argument, so the call queues no host-to-device copy and returns
 * without waiting for the device.
 * pixels: device pool [n_pixels][3]; flags: device [n_pixels] (DT_FLAG_* of
 * each pixel's ray tree, as dt_trace_forward's) or NULL; path_sig: device
 * [n_pixels] (dt_trace_forward's path signature of each pixel) or NULL.  An
 * admitted request's pixel range in all three is cleared by its admitting
 * step, then accumulated into.
 * slot_live: device [DT_SERVE_MAX_SLOTS], overwritten with each slot's live
 * rays after the step.  slot_dropped: device [DT_SERVE_MAX_SLOTS], each
 * slot's rays lost to a full queue since the slot's request was admitted
 * (cleared by the admitting step): a request that finishes with a nonzero
 * count has an incomplete image, and its pixels carry DT_FLAG_OVERFLOW where
 * flags is given.  stats: device int64 [3] or NULL: rays traced since reset,
 * rays dropped since reset, live rays.  step: 0, 1, 2, ... since the reset
 * (selects the queue buffer). */
dt_status dt_serve_step(const dt_serve_scene* scenes, int32_t n_scenes, const dt_env* envs,
                        int32_t n_envs, const dt_serve_admit* admits, int32_t n_admits,
                        int64_t step, float* pixels, int32_t* flags, uint64_t* path_sig,
                        int64_t n_pixels, uint32_t* slot_live, uint32_t* slot_dropped,
                        int64_t* stats, int64_t queue_capacity, float t_eps, void* ws,
                        size_t ws_bytes, void* stream);

/* Closest hit of n rays (o, d [n][3], skip [n] = triangle to ignore or -1,
 * may be NULL) with t > t_eps; ties in t go to the smaller triangle id.
 * Outputs tri [n] (-1 = miss), t [n], b [n][2] (weights of v1 and v2).
 * brute_force = 1 tests every triangle with the same predicate. */
dt_status dt_intersect(const dt_scene* sc, const float* o, const float* d, const int32_t* skip,
                       int64_t n, float t_eps, int32_t brute_force, int32_t* tri, float* t,
                       float* b, void* stream);

const char* dt_status_string(dt_status s);
const char* dt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DIFFTRANS_H */
