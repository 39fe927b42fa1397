/*
 * ipt.h -- C ABI of the MI355X (gfx950) inverse path tracing library.
 *
 * The library implements the hot path of "Inverse Path Tracing for Joint
 * Material and Lighting Estimation" (Azinovic et al., CVPR 2019): a Monte
 * Carlo path tracer whose image estimate (Sec. 3.1, Eq. 1-2) and whose
 * gradient with respect to per-object material and emission unknowns
 * (Sec. 3.3, Eq. 4-6) are nested inside stochastic gradient descent
 * (Sec. 3.2, Eq. 3; Sec. 4.5).
 *
 * Conventions shared by every call:
 *   - Unless stated otherwise, pointers to arrays are DEVICE pointers (HIP
 *     global memory on the device that is current when the call is made);
 *     the caller owns them and the library never frees them.  Scene inputs of
 *     ipt_scene_build are HOST pointers (copied).
 *   - hip_stream is a hipStream_t (NULL = the default stream).  All device
 *     work is enqueued on it; no call synchronises the stream except
 *     ipt_scene_build and ipt_scene_info.
 *   - Every call returns an ipt_status and never aborts.  Arguments are
 *     validated on the host before anything is enqueued; on error nothing is
 *     enqueued and ipt_last_error() returns a message (thread-local).
 *   - The library allocates device memory only in ipt_scene_build,
 *     ipt_guide_create and the first ipt_guide_cache_build call of a guide on
 *     a scene (or with a new cell area); all of it is owned by the handle and
 *     freed by the matching _free.  Per-call scratch space is the caller's
 *     workspace.
 *
 * Parameter vector (float32, raw physical values, length P = M S + 3 E with
 * M material parameters per segment, fixed per scene by ipt_build_opts):
 *   segment s   [M s .. M s + M-1]  material parameters of the segment
 *   emitter k   [M S+3k .. +2]      e_r e_g e_b (radiance of segment emitter_seg[k])
 * Material models (Sec. 3.3 material unknowns, Sec. 4.1):
 *   IPT_MATERIAL_GGX (M = 7, the default): kd_r kd_g kd_b ks_r ks_g ks_b alpha;
 *     f = kd/pi + ks D(h) G1(o) G1(i) / (4 cos_o cos_i), GGX D with alpha
 *     clamped to [1e-3, 1], separable Smith G1, no Fresnel.
 *   IPT_MATERIAL_DISNEY (M = 13): the Disney model of Sec. 4.1 (Burley
 *     2012): base_r base_g base_b subsurface metallic specular specular_tint
 *     roughness anisotropic sheen sheen_tint clearcoat clearcoat_gloss, each
 *     meant for [0, 1] (the caller's Adam bounds keep them there).  Its
 *     anisotropy uses a tangent frame per vertex: the hit triangle's first edge
 *     (vertex 1 - vertex 0) projected onto the shading plane.
 * Emission: constant radiance e, or the profile e (w.n)_+ of Sec. 4.3
 * (emission_profile = 1); emitters emit on the side their triangle winding
 * faces.
 *
 * Random numbers: Philox4x32-10, key = (seed_lo ^ stream_tag*0x9E3779B9,
 * seed_hi), counter = (path_lo, path_hi, 2*vertex + half, iteration), uniform
 * = (x >> 8) * 2^-24.  path id = pixel * spp + sample, pixel =
 * (view * height + y) * width + x (row 0 is the top row).  Identical inputs
 * give identical paths, which is what lets the adjoint pass replay them.
 */
#ifndef IPT_H
#define IPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipt_scene_s *ipt_scene_t;
typedef struct ipt_guide_s *ipt_guide_t;

typedef enum {
    IPT_OK = 0,
    IPT_ERR_INVALID_ARG = 1,
    IPT_ERR_BAD_SCENE = 2,
    IPT_ERR_OUT_OF_MEMORY = 3,
    IPT_ERR_WORKSPACE_TOO_SMALL = 4,
    IPT_ERR_HIP = 5,
    IPT_ERR_NOT_SUPPORTED = 6
} ipt_status;

/* Pinhole cameras (Sec. 3.4: several calibrated views).  cam_to_world is a
 * DEVICE array [num_views][4][4] (row-major, acting on column vectors; the
 * camera looks down its -z axis, +y up); fov_y is a DEVICE array
 * [num_views] of vertical fields of view in radians. */
typedef struct {
    int32_t num_views, width, height;
    const float *cam_to_world;
    const float *fov_y;
} ipt_cameras;

/* One estimator configuration (one "stream" of independent samples). */
typedef struct {
    uint64_t seed;
    uint32_t stream_tag;      /* 0 target, 1 colour (A), 2 gradient (B), 3 guide */
    uint32_t iteration;       /* SGD iteration: fresh samples every step */
    int32_t spp;              /* samples per pixel, >= 1 */
    int32_t max_depth;        /* D: scattering vertices per path, 1..16 */
    int32_t rr_depth;         /* Russian roulette at vertices >= rr_depth; < 0 off */
    int32_t mis;              /* 0 BRDF only, 1 light only, 2 balance, 3 power heuristic */
    int32_t emission_profile; /* 0 constant radiance, 1 e (w.n)_+ */
    int32_t jitter;           /* 1 box pixel filter, 0 pixel centres */
    int32_t replay_traverse;  /* gradient only: 1 = adjoint re-traces rays instead of
                                 reading vertex checkpoints */
    const int64_t *pixel_list;/* DEVICE [num_pixels] or NULL = every pixel of every view */
    int64_t num_pixels;
    ipt_guide_t guide;        /* NULL = BRDF sampling only */
    float guide_mix;          /* probability of sampling the guide when guide != NULL */
    int32_t guide_fp32;       /* 1: evaluate the guide in float32 on VALU (reference
                                 mode) instead of bfloat16 MFMA */
    uint64_t *debug_path_hash;/* DEVICE [pixels*spp] or NULL: FNV-1a of each path's events */
    const uint8_t *path_mask; /* DEVICE [pixels*spp] or NULL: 0 removes the path */
    float *debug_path_radiance;/* DEVICE [pixels*spp][3] or NULL (ipt_render only) */
    float *debug_vertices;    /* DEVICE [pixels*spp][max_depth+1][8] or NULL (ipt_render
                                 only): per vertex input triangle id, u, v, t and the
                                 path radiance accumulated so far */
    int32_t guide_cached;     /* 1: sample the guide's cached proposal (rows built by
                                 ipt_guide_cache_build for this scene) instead of
                                 evaluating the network at every vertex; 0: per vertex */
} ipt_render_opts;

typedef struct {
    float lr, beta1, beta2, eps;
} ipt_adam_opts;

typedef struct {
    int64_t num_triangles, num_vertices, num_nodes, num_light_triangles;
    int32_t num_segments, num_emitters, bvh_depth, has_normals;
                              /* bvh_depth: levels of the binary SAH tree (the
                                 four-child tree of the traversal has about 60% as many or fewer) */
    double sah_cost;          /* SAH cost of the BVH (C_trav = C_isect = 1) */
    double build_ms;          /* wall time of the BVH build */
    float scene_diag;
    uint64_t nonfinite_paths; /* paths dropped for a non-finite contribution */
    uint64_t stack_overflows; /* traversals that ran out of stack */
    int32_t bvh_builder;      /* the ipt_bvh_builder that built the BVH */
    int32_t params_global;    /* 1: parameters in global memory (ipt_param_storage) */
    int32_t node_bytes;       /* bytes per BVH node of the traversal (64: 4-wide with quantized
                                 child boxes, the default, or binary; 128: 4-wide with float
                                 boxes); num_nodes counts these nodes */
    int32_t material_model;   /* the ipt_material_model of the scene */
    int32_t params_per_segment; /* M: 7 or 13 */
    int32_t node_width;       /* children per BVH node of the traversal: 4 or 2 */
} ipt_scene_info_t;

/* Where the BVH is built.  Both builders apply the same rule (binned SAH,
 * 64 slabs per axis, C_trav = C_isect = 1, leaves of at most 2 triangles)
 * and give the same tree; the host builder is kept as a reference. */
typedef enum { IPT_BVH_GPU = 0, IPT_BVH_HOST = 1 } ipt_bvh_builder;
/* Where the path kernels keep the parameter vector (M S + 3 E floats) and
 * the adjoint its gradient.  LDS: a copy per block and per-block float64
 * partial gradients summed in a fixed order (deterministic).  GLOBAL: read
 * through the caches, and the adjoint adds float64 atomics into R replicas of
 * the gradient (block b into replica b mod R, R bounded by 256 MB of
 * workspace), summed in a fixed order afterwards (summation order within a
 * replica varies; for many segments, e.g. one per triangle, where contention
 * is low).  AUTO: LDS up to 4096 parameters. */
typedef enum { IPT_PARAMS_AUTO = 0, IPT_PARAMS_GLOBAL = 1 } ipt_param_storage;
/* The material model of every segment of a scene (see the parameter vector
 * above); any other value is IPT_ERR_INVALID_ARG. */
typedef enum { IPT_MATERIAL_GGX = 0, IPT_MATERIAL_DISNEY = 1 } ipt_material_model;
typedef struct {
    int32_t bvh_builder;      /* an ipt_bvh_builder */
    int32_t param_storage;    /* an ipt_param_storage */
    int32_t material_model;   /* an ipt_material_model */
} ipt_build_opts;

/* Build a scene: upload geometry, build the BVH on the GPU (binned SAH,
 * leaves of at most 2 triangles), the leaf-ordered triangle layout and the
 * emitter table, all on hip_stream (the call synchronises it).
 * Inputs are HOST arrays: verts [nv][3], normals [nv][3] or NULL (flat
 * shading), tris [nt][3] vertex indices, tri_seg [nt] segment ids in
 * [0, num_segments), emitter_seg [num_emitters] distinct segment ids.  The
 * triangles of an emitter segment emit; every segment reflects.
 * Sec. 4.2 (per-vertex normals, per-object constant parameters).
 * Errors: IPT_ERR_INVALID_ARG (NULL/size), IPT_ERR_BAD_SCENE (index out of
 * range, non-finite vertex or one with a coordinate beyond 1e12 in
 * magnitude, degenerate emitter triangle, duplicate emitter),
 * IPT_ERR_NOT_SUPPORTED (more than 2^27 triangles, or a BVH deeper than the
 * traversal stack), IPT_ERR_OUT_OF_MEMORY / IPT_ERR_HIP (device). */
ipt_status ipt_scene_build(const float *verts, int64_t nv, const float *normals,
                           const int32_t *tris, const int32_t *tri_seg, int64_t nt,
                           int32_t num_segments, const int32_t *emitter_seg,
                           int32_t num_emitters, void *hip_stream, ipt_scene_t *out);
/* ipt_scene_build with build options (NULL = defaults: GPU builder). */
ipt_status ipt_scene_build_ex(const float *verts, int64_t nv, const float *normals,
                              const int32_t *tris, const int32_t *tri_seg, int64_t nt,
                              int32_t num_segments, const int32_t *emitter_seg,
                              int32_t num_emitters, const ipt_build_opts *opts,
                              void *hip_stream, ipt_scene_t *out);
ipt_status ipt_scene_free(ipt_scene_t scene);
/* Sizes, BVH statistics and device error counters (synchronises). */
ipt_status ipt_scene_info(ipt_scene_t scene, ipt_scene_info_t *out);

/* Workspace bytes for ipt_render / ipt_render_grad / ipt_loss_grad with these
 * options: *min_bytes lets the gradient run in chunks; *full_bytes keeps the
 * vertex checkpoints of every gradient path at once. */
ipt_status ipt_workspace_query(ipt_scene_t scene, const ipt_cameras *cams,
                               const ipt_render_opts *opts, size_t *min_bytes,
                               size_t *full_bytes);

/* Image estimate (Sec. 3.1, Eq. 1): image [pixels][3] float32 receives the
 * mean over spp of each path's radiance.  params [P] are the values to
 * render with; sampling_params [P] (NULL = params) fix every sampling
 * decision, pdf, MIS weight and the light-selection distribution. */
ipt_status ipt_render(ipt_scene_t scene, const ipt_cameras *cams, const float *params,
                      const float *sampling_params, const ipt_render_opts *opts, float *image,
                      void *workspace, size_t workspace_bytes, void *hip_stream);

/* ipt_render for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same image estimate with no workspace argument.  Its scratch (work counter,
 * light-selection table, traversal overflow stacks, per-chunk sample sums)
 * is a fixed 40 MiB device array inside the library, one per device, held
 * until the process ends; the call allocates nothing, host or device, and
 * launches at most 2 blocks per CU of the colour kernel.  All calls on one
 * device share that array, so calls that overlap on one device (concurrent
 * streams, threads) race and must be serialised by the caller.  Inputs and
 * outputs as for ipt_render (the debug outputs of opts included).  Errors:
 * as ipt_render, plus IPT_ERR_NOT_SUPPORTED when the scratch would exceed
 * 40 MiB (25 MiB of overflow stacks, up to 4.5 MiB of per-chunk sums and 8 B
 * per light triangle: scenes of more than about 1.4 million light
 * triangles) and IPT_ERR_INVALID_ARG when the scene was built on another
 * device than the current one. */
ipt_status ipt_render_static(ipt_scene_t scene, const ipt_cameras *cams, const float *params,
                             const float *sampling_params, const ipt_render_opts *opts, float *image,
                             void *hip_stream);

/* Vector-Jacobian product of the image estimate (Sec. 3.3, Eq. 5-6):
 * grad [P] = sum_j sum_c w[j][c] d I_jc / d theta, with w [pixels][3] the
 * adjoint image.  The estimate uses the samples of opts (stream B); pdfs are
 * held at sampling_params.  The forward pass stores per-vertex checkpoints and
 * the division-free suffix radiance; the adjoint pass replays each path from
 * its Philox counter.  grad is overwritten. */
ipt_status ipt_render_grad(ipt_scene_t scene, const ipt_cameras *cams, const float *params,
                           const float *sampling_params, const ipt_render_opts *opts,
                           const float *w, float *grad, void *workspace,
                           size_t workspace_bytes, void *hip_stream);

/* One SGD evaluation (Sec. 3.2-3.3): render the colour estimate with
 * color_opts, form the loss against target [pixels][3] (loss_kind 0: mean
 * squared error over pixels and channels; 1: mean absolute error, Eq. 3) and
 * its adjoint dE/dI, then the gradient from independent samples (grad_opts,
 * Sec. 3.3: the two estimates must be independent).  loss: DEVICE scalar.
 * image_A [pixels][3] (nullable) receives the colour estimate. */
ipt_status ipt_loss_grad(ipt_scene_t scene, const ipt_cameras *cams, const float *params,
                         const float *target, const ipt_render_opts *color_opts,
                         const ipt_render_opts *grad_opts, int32_t loss_kind, float *loss,
                         float *grad, float *image_A, void *workspace, size_t workspace_bytes,
                         void *hip_stream);

/* Adam (Sec. 4.5) on theta = params/scale with bias correction (step >= 1),
 * then theta is clamped to [lo, hi].  m, v [P] are the moment buffers
 * (theta units).  scale/lo/hi/trainable may be NULL (1, -inf, +inf, all). */
ipt_status ipt_sgd_step(float *params, const float *grad, float *m, float *v, int32_t P,
                        int32_t step, const ipt_adam_opts *adam, const float *scale,
                        const float *lo, const float *hi, const uint8_t *trainable,
                        void *hip_stream);

/* L1 regulariser of the emission (Sec. 4.4, "Regularization"; App. E: an
 * L1 term on all emission parameters, since most objects emit nothing):
 * grad[i] += weight[i] * sgn(params[i]) and *loss += sum_i weight[i] |params[i]|,
 * with sgn(0) = 0.  params, grad, weight [P] and loss [1] are DEVICE float32
 * arrays; weight is 0 for the entries that are not regularised.  Call it
 * after ipt_loss_grad and before ipt_sgd_step.  Errors: IPT_ERR_INVALID_ARG
 * (NULL pointer, P < 1). */
ipt_status ipt_l1_reg(const float *params, float *grad, const float *weight, int32_t P, float *loss,
                      void *hip_stream);

/* Closest hits of a batch of rays (the ray-casting step of every path
 * vertex).  origins/dirs [n][3]; out_tri [n] original triangle id or -1;
 * out_tuv [n][3] (t, u, v) with u, v the weights of vertices 1 and 2;
 * skip_tri [n] (nullable) excludes one triangle per ray; brute_force = 1
 * tests every triangle (checks the BVH).  Ties in t go to the smaller id. */
ipt_status ipt_trace_rays(ipt_scene_t scene, const float *origins, const float *dirs,
                          const int32_t *skip_tri, int64_t n, float tmin, int32_t brute_force,
                          int32_t *out_tri, float *out_tuv, void *hip_stream);

/* Learned path-guiding proposal: an MLP (bfloat16 MFMA inference and
 * training, float32 accumulation and master weights) that maps a path
 * vertex -- position normalised to the scene box, shading normal, outgoing
 * direction -- and a learned 16-d embedding of its segment to an 8-lobe von
 * Mises-Fisher mixture over incident directions, trained towards the
 * product of BRDF, cosine and incident radiance.  Attached to
 * ipt_render_opts.guide with guide_mix = c > 0, every continuation direction
 * is drawn from the mixture with probability c and from the BRDF otherwise,
 * and weighted by the combined density c q + (1 - c) p_brdf (one-sample MIS),
 * so every estimate stays unbiased; c = 0 samples the BRDF only.  A guide
 * attached to the gradient pass (ipt_render_grad / ipt_loss_grad) also makes
 * that pass write training records (vertex features, sampled direction,
 * estimate of BRDF x cosine x incident radiance over the sampling density)
 * for every record_stride-th path into the guide's ring.  The guide does not depend on the unknowns and is not
 * differentiated.  Not part of the paper's method (Sec. 3.1 uses BRDF and
 * light sampling); the estimator it feeds is the paper's. */
typedef struct {
    uint64_t seed;          /* initial weights */
    float lr;               /* Adam learning rate of the network and embedding */
    int32_t batch;          /* training records per step (multiple of 64) */
    int32_t ring_capacity;  /* training records kept */
    int32_t record_stride;  /* record every record_stride-th gradient path */
} ipt_guide_opts;

/* Allocates the network, its Adam state and the record ring (the library
 * owns them).  The scene fixes the segment count and the box. */
ipt_status ipt_guide_create(ipt_scene_t scene, const ipt_guide_opts *opts, void *hip_stream,
                            ipt_guide_t *out);
ipt_status ipt_guide_free(ipt_guide_t guide);
/* Cached proposal: the network evaluated once per surface cell and side
 * instead of at every path vertex.  Every triangle's barycentric domain is cut
 * into n^2 sub-triangles (grid squares of side 1/n in (u, v), each halved by
 * its anti-diagonal), n the smallest integer in [1, 64] with
 * |e1 x e2| <= 2 n^2 cell_area (decided in float32: squares compared, fixed
 * operation order, no contraction).  A cell's query is its centroid, the
 * shading normal there (negated for the back side) and an outgoing direction
 * along that normal.  With ipt_render_opts.guide_cached = 1 a path vertex
 * samples and weights with the row of the cell and side it hit, so the
 * estimator stays unbiased (the proposal is any density; only the density it
 * was sampled from enters the weights).  The first call for a scene, or with a
 * new cell_area, allocates the cell table and the rows (192 B per cell and
 * side; at most 2^24 cells per side, else IPT_ERR_INVALID_ARG) and
 * synchronises the stream once; later calls only refill the rows from the
 * current weights and allocate nothing.  mode 0: bfloat16 MFMA network, 1:
 * float32 VALU (reference).  *num_cells (HOST, nullable): cells per side.
 * Rebuild after training steps; rows are read by the render calls on the
 * same stream.  Not part of the paper's method. */
ipt_status ipt_guide_cache_build(ipt_guide_t guide, ipt_scene_t scene, float cell_area, int32_t mode,
                                 int64_t *num_cells, void *hip_stream);
/* Mixture for n queries: feat [n][9] (DEVICE: normalised position, normal,
 * outgoing direction), seg [n] (DEVICE); out [n][40] (DEVICE) = per lobe
 * (mu xyz, kappa, weight).  mode 0: bfloat16 MFMA, 1: float32 VALU. */
ipt_status ipt_guide_eval(ipt_guide_t guide, const float *feat, const int32_t *seg, int64_t n,
                          int32_t mode, float *out, void *hip_stream);
/* steps Adam steps on minibatches drawn from the ring; *loss_out (HOST,
 * nullable) receives the last batch's loss (synchronises when given). */
ipt_status ipt_guide_train(ipt_guide_t guide, int32_t steps, float *loss_out, void *hip_stream);
/* Copy the float32 parameters (16744 network values then 16 per segment)
 * to (get = 1) or from (get = 0) the HOST array w; synchronises. */
ipt_status ipt_guide_weights(ipt_guide_t guide, float *w, int32_t get, int64_t count);
/* Number of records written so far (the ring keeps the last capacity; the
 * count is 32-bit and wraps after 2^32 records). */
ipt_status ipt_guide_records(ipt_guide_t guide, int64_t *count);
/* Training record, 16 float32 (the ring's layout):
 *   [0..2]  position normalised to the scene box, [3] segment (int32 bits),
 *   [4..6]  shading normal (facing the outgoing side), [7] weight L/p,
 *   [8..10] outgoing direction, [11] path index (int32 bits),
 *   [12..14] sampled incident direction, [15] vertex index k >= 1 (int32 bits).
 * The weight is the luminance of f cos L_i / p: the BRDF times the cosine
 * times the radiance estimate arriving along the sampled direction, over
 * the combined density it was sampled with (the training target is the
 * product f cos L_i, which vanishes below the surface). */
/* Loss -sum_i w_i log q_i / sum_i w_i of n records rec [n][16] (DEVICE), and
 * its gradient grad [16744 + 16 S] (DEVICE) with respect to the float32
 * parameters, through the bfloat16 forward pass; *loss is DEVICE.  Does not
 * change the guide.  1 <= n <= 2^24. */
ipt_status ipt_guide_loss_grad(ipt_guide_t guide, const float *rec, int64_t n, float *loss, float *grad,
                               void *hip_stream);
/* Appends n records rec [n][16] (DEVICE) to the ring (0 <= n <= capacity). */
ipt_status ipt_guide_add_records(ipt_guide_t guide, const float *rec, int64_t n, void *hip_stream);
/* Copies ring slots [0, n) to out [n][16] (DEVICE); 0 <= n <= capacity.
 * Slot i holds record i mod capacity of the order in which records arrived
 * (for records from a gradient pass that order is not deterministic). */
ipt_status ipt_guide_read_records(ipt_guide_t guide, float *out, int64_t n, void *hip_stream);

/* Kernel timing and work counters of the path kernels of one scene (kernel
 * 0: colour pass, 1: gradient forward pass, 2: adjoint replay).  While
 * enabled, every launch is bracketed by HIP events on the stream it is
 * launched on, and the kernels add their work (rays cast, BVH nodes fetched,
 * triangles tested, paths, path vertices, work units) into per-scene device
 * counters.  A work unit is one pixel with all its samples when there are at
 * least two pixels per lane of the grid (a lane then walks every sample of
 * its pixel and forms the mean in registers), else a chunk of a pixel's
 * samples; units == pixels means the first mode.
 * ipt_profile_read synchronises the device; ipt_profile_reset clears both. */
typedef struct {
    int64_t launches;
    double total_ms;          /* sum of event-measured launch durations */
    uint64_t rays, nodes, tris, paths, vertices, units;
} ipt_kernel_profile;

ipt_status ipt_profile_enable(ipt_scene_t scene, int32_t enable);
ipt_status ipt_profile_read(ipt_scene_t scene, int32_t kernel, ipt_kernel_profile *out);
ipt_status ipt_profile_reset(ipt_scene_t scene);

const char *ipt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IPT_H */
