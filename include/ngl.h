/*
 * ngl.h -- C ABI of the MI355X (gfx950) neural geometric LOD library.
 *
 * The library evaluates a neural signed distance function stored as a
 * sparse voxel octree of corner feature vectors (Takikawa et al., "Neural
 * Geometric Level of Detail", arXiv 2101.10994, Sec. 3.2) and sphere-traces
 * rays through it (Sec. 3.4).  Entry points follow the paper's statement of
 * the problem: build the octree from occupancy, query the SDF at a discrete
 * or continuous LOD, trace rays, take a training step.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Feature level l (1-based, l = 1..L) has grid resolution 4 * 2^(l-1)
 *    and lives at octree depth l+1; depth d has resolution 2^d; the root
 *    (depth 0) is the box [-1,1]^3 (App. A.1: the rendering octree starts at
 *    1^3, features start at resolution 4).
 *  - Canonical layout: at every depth voxels are numbered by increasing
 *    Morton code (bit 3k = x, 3k+1 = y, 3k+2 = z); corners of a feature level
 *    by the Morton code of their lattice point.  Child c of a voxel is cell
 *    2*ijk + (c&1, c>>1&1, c>>2&1); corner slot j of a voxel is lattice
 *    point ijk + (j&1, j>>1&1, j>>2&1).
 *  - Points and rays are structure-of-arrays float32: x[3][P] means the P
 *    x-coordinates, then the P y's, then the P z's.
 *  - Pointers named "device" must point to GPU memory (any hipMalloc'd or
 *    torch allocation on the current device); "host" pointers to CPU memory.
 *    The caller owns every buffer; the library never allocates or frees
 *    device memory and never synchronises the stream except where stated.
 *  - `stream` is a hipStream_t (NULL = the null stream); all GPU work of a
 *    call is enqueued on it in order.
 *  - Every function returns an ngl_status; nothing throws across the ABI.
 *    On error, ngl_last_error() returns a thread-local description.
 *    Per-point and per-ray outcomes (a point outside the octree, a ray that
 *    misses) are data, not errors.
 */
#ifndef NGL_H
#define NGL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NGL_MAX_LODS 8
#define NGL_MAX_DEPTH (NGL_MAX_LODS + 2)
#define NGL_MAX_FEAT_DIM 64
#define NGL_MAX_HIDDEN 256

typedef enum {
  NGL_OK = 0,
  NGL_E_INVALID = 1,     /* bad argument (null pointer, size, lod, dtype) */
  NGL_E_CAPACITY = 2,    /* a caller-sized buffer is too small; see the call */
  NGL_E_HIP = 3,         /* a HIP runtime call failed */
  NGL_E_UNSUPPORTED = 4  /* valid but unsupported combination */
} ngl_status;

typedef enum { NGL_F32 = 0, NGL_F16 = 1, NGL_BF16 = 2 } ngl_dtype;

/* Per-ray outcome of ngl_sphere_trace. */
typedef enum {
  NGL_RAY_MISS = 0,      /* ran out of voxels along the ray */
  NGL_RAY_HIT = 1,       /* SDF fell below the hit threshold */
  NGL_RAY_MAX_STEPS = 2, /* step budget exhausted */
  NGL_RAY_FAR = 3,       /* passed the far plane */
  NGL_RAY_STALLED = 4,   /* oscillation rule fired (only if enabled) */
  NGL_RAY_INVALID = 5    /* non-finite origin or direction */
} ngl_ray_status;

const char* ngl_status_str(int status);
const char* ngl_last_error(void);
int ngl_version(void);

/* Process-wide implementation choices (they never change results beyond
 * the stated tolerances; the autotuner sets them).
 *  NGL_OPT_F32_DECODER: how the decoder's first layer runs for FP32
 *    weights: 0 = per lane on the vector ALUs with weights read through the
 *    scalar cache, 1 = on the matrix cores (v_mfma_f32_16x16x4f32, FP32
 *    operands and accumulation; default).
 *  NGL_OPT_TRACE_WAVES: wavefronts per block of the matrix-core tracers
 *    (1, 2 or 4; 0 = the most that fit in 64 KB of LDS, default).
 *  NGL_OPT_TRACE_BLOCKS_PER_CU: cap on resident tracer blocks per compute
 *    unit (0 = occupancy limit, default), applied to every persistent
 *    tracer launch (one-lane and lanes-per-ray phases, batched views, LOD
 *    groups).
 *  NGL_OPT_TRACE_PAUSE1, NGL_OPT_TRACE_PAUSE2: evaluation counts at which
 *    a phased ngl_sphere_trace parks the rays still running (0..4096, 0 =
 *    no such phase; a second count not above the first is ignored).
 *  NGL_OPT_TRACE_WIDE: 1 (default) = the last phase of a phased trace
 *    serves each ray with a group of lanes (matrix-core decoders only),
 *    0 = one lane per ray throughout.
 *  NGL_OPT_COOP_GATHER: 1 (default) = the matrix-core query and normal
 *    kernels gather each feature row with a group of lanes, each holding a
 *    slice of it, 0 = one lane per point reads whole rows (same results).
 *  NGL_OPT_QUERY_BLOCKS_PER_CU: blocks per compute unit of the
 *    cooperative query kernel, whose blocks loop over the points (0..64;
 *    0 = as many as are resident at once, default).
 * NGL_E_INVALID for an unknown option or value. */
typedef enum {
  NGL_OPT_F32_DECODER = 0,
  NGL_OPT_TRACE_WAVES = 1,
  NGL_OPT_TRACE_BLOCKS_PER_CU = 2,
  NGL_OPT_TRACE_PAUSE1 = 3,
  NGL_OPT_TRACE_PAUSE2 = 4,
  NGL_OPT_TRACE_WIDE = 5,
  NGL_OPT_COOP_GATHER = 6,
  NGL_OPT_QUERY_BLOCKS_PER_CU = 7,
  NGL_OPT_COUNT = 8
} ngl_option;
int ngl_set_option(int option, int value);
int ngl_get_option(int option, int* value);

/* ------------------------------------------------------------------ */
/* 1. Octree from occupancy (Sec. 3.2: a voxel exists only where there   */
/*    is surface; Sec. 3.4: parents always exist, and the voxel-to-corner */
/*    pointers are precomputed in an initialisation pass).  Host-side.    */
/* ------------------------------------------------------------------ */

/* Sizes of the octree built from `n` occupied finest cells ijk[n][3]
 * (host, int32, each coordinate in [0, 2^(num_lods+1))), duplicates allowed.
 * Depth-d voxels are the parent closure {cell >> (D-d)}, D = num_lods+1.
 * Writes nvox[num_lods+2] (voxels per depth 0..D) and ncorner[num_lods]
 * (distinct corner lattice points per feature level), both host.
 * NGL_E_INVALID if num_lods is outside 1..NGL_MAX_LODS or a cell is out of
 * range. */
int ngl_octree_plan(const int32_t* ijk, int64_t n, int32_t num_lods, int64_t* nvox, int64_t* ncorner);

/* Host output buffers of ngl_octree_fill, sized from ngl_octree_plan.
 * Index d is a depth (0..D), index l-1 a feature level l (1..num_lods).
 * Any pointer may be NULL to skip that array. */
typedef struct {
  uint32_t* cell[NGL_MAX_DEPTH];        /* [nvox[d]] packed cell x | y<<10 | z<<20 */
  uint8_t* child_mask[NGL_MAX_DEPTH];   /* [nvox[d]] bit c set iff child c exists */
  int32_t* first_child[NGL_MAX_DEPTH];  /* [nvox[d]] index of the first child at d+1 (-1: none) */
  int32_t* parent[NGL_MAX_DEPTH];       /* [nvox[d]] index of the parent at d-1 (-1 at the root) */
  int32_t* corners[NGL_MAX_LODS];       /* [nvox[l+1]][8] corner index of slot j */
  int32_t* corner_cell[NGL_MAX_LODS];   /* [ncorner[l-1]][3] lattice point of each corner */
  int32_t* corner_adj_off[NGL_MAX_LODS]; /* [ncorner[l-1]+1] CSR offsets into corner_adj */
  int32_t* corner_adj[NGL_MAX_LODS];     /* [8*nvox[l+1]] 8*v+j of every (voxel, slot) using the
                                            corner, ascending per corner (used by training) */
} ngl_octree_host;

/* Fill the canonical layout (same inputs as ngl_octree_plan). */
int ngl_octree_fill(const int32_t* ijk, int64_t n, int32_t num_lods, const ngl_octree_host* out);

/* The same build on the device, bit for bit the arrays of ngl_octree_fill,
 * without host synchronisation: ijk is device int32 [n][3]; the arrays are
 * device buffers allocated to upper bounds (depth d: min(n, 8^d) voxels,
 * at least 1; level l: 8 * (voxels of depth l+1) corner slots, corners and
 * adjacency entries, corner_adj_off one more); the actual sizes are written
 * to nvox (device [num_lods+2]) and ncorner (device [num_lods]), and the
 * number of cells outside [0, 2^(num_lods+1))^3 (which are skipped) to
 * *bad (device).  cell/parent are required at every depth, child_mask and
 * first_child at depths 0..num_lods (optional at num_lods+1: mask 0, first
 * child -1), corners at every level; corner_cell and the adjacency pair are
 * optional.  n < 2^28.  ws: device bytes from
 * ngl_octree_build_device_workspace(n, num_lods). */
typedef struct {
  uint32_t* cell[NGL_MAX_DEPTH];
  uint8_t* child_mask[NGL_MAX_DEPTH];
  int32_t* first_child[NGL_MAX_DEPTH];
  int32_t* parent[NGL_MAX_DEPTH];
  int32_t* corners[NGL_MAX_LODS];
  int32_t* corner_cell[NGL_MAX_LODS];
  int32_t* corner_adj_off[NGL_MAX_LODS];
  int32_t* corner_adj[NGL_MAX_LODS];
  int64_t* nvox;    /* device [num_lods + 2] */
  int64_t* ncorner; /* device [num_lods] */
  int64_t* bad;     /* device [1] */
} ngl_octree_device;
int ngl_octree_build_device_workspace(int64_t n, int32_t num_lods, size_t* bytes);
int ngl_octree_build_device(const int32_t* ijk, int64_t n, int32_t num_lods, const ngl_octree_device* out,
                            void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* Device view of a model: octree + corner features + per-LOD decoders.  */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t num_lods;   /* L: feature levels, 1..NGL_MAX_LODS (octree depth L+1) */
  int32_t feat_dim;   /* m: feature width, multiple of 8, <= NGL_MAX_FEAT_DIM */
  int32_t hidden;     /* h: decoder hidden width, multiple of 16, <= NGL_MAX_HIDDEN */
  int32_t with_xyz;   /* 1: decoder input is [x, y, z, z_0..z_{m-1}] (Eq. 2); 0: [z] */
  int32_t feat_dtype; /* ngl_dtype of feat[] (F32, F16 or BF16) */
  int32_t w_dtype;    /* ngl_dtype of W1[] (F32 or BF16); b1, w2, b2 are always F32 */
  int64_t nvox[NGL_MAX_DEPTH];               /* voxels per depth 0..L+1 */
  int64_t ncorner[NGL_MAX_LODS];             /* corners per level */
  const uint32_t* cell[NGL_MAX_DEPTH];       /* device, packed cells per depth */
  const uint8_t* child_mask[NGL_MAX_DEPTH];  /* device, depths 0..L */
  const int32_t* first_child[NGL_MAX_DEPTH]; /* device, depths 0..L */
  const int32_t* parent[NGL_MAX_DEPTH];      /* device, depths 1..L+1 */
  const int32_t* corners[NGL_MAX_LODS];      /* device, [nvox[l+1]][8], 16-byte aligned */
  const void* feat[NGL_MAX_LODS];            /* device, [ncorner[l-1]][m], feat_dtype; 16-byte aligned, below 4 GiB per level */
  const void* W1[NGL_MAX_LODS];              /* device, [h][din] row-major, w_dtype */
  const float* b1[NGL_MAX_LODS];             /* device, [h] */
  const float* w2[NGL_MAX_LODS];             /* device, [h] */
  const float* b2;                           /* device, [L] */
  const int32_t* corner_adj_off[NGL_MAX_LODS]; /* device, training only: CSR of corner -> 8*v+j */
  const int32_t* corner_adj[NGL_MAX_LODS];
  /* device, nullable: decoder l's first layer [W1 | b1] pre-packed by
   * ngl_pack_decoders in the fragment order of the matrix-core decoder; when
   * set, kernels copy it instead of rebuilding the fragments from W1 and b1
   * in every block.  Must be re-packed whenever W1 or b1 change. */
  const void* W1_packed[NGL_MAX_LODS];
} ngl_model;

/* Decoder weights in matrix-core fragment order (Eq. 2's first layer,
 * Sec. 4.1's 35 -> h -> 1 decoder).  For BF16 weights (w_dtype NGL_BF16) the
 * fragments of v_mfma_f32_16x16x32_bf16: per hidden tile of 16 rows, one
 * 32-column feature step per 32 features, then one step holding
 * [W1_x, W1_x, b1_hi, b1_lo] (the position weights twice, for the high and
 * low parts of x, and b1 split into two BF16 values); for FP32 weights the
 * fragments of v_mfma_f32_16x16x4f32 over [W1 | b1].  Each lane's part of a
 * fragment is stored contiguously (16 bytes for BF16, 4 for FP32), 64 lanes
 * per fragment.
 * ngl_packed_decoder_bytes: bytes for all num_lods decoders (a multiple of
 * 256 per LOD).  ngl_pack_decoders writes them into `packed` (device,
 * 256-byte aligned, at least that many bytes, caller-owned) and sets
 * m->W1_packed[l] to decoder l+1's part.  The packed form does not depend on
 * NGL_OPT_F32_DECODER (the per-lane FP32 form ignores it).
 * Errors: NGL_E_INVALID for a bad model, null or misaligned buffer, or too
 * few bytes. */
int ngl_packed_decoder_bytes(const ngl_model* m, size_t* bytes);
int ngl_pack_decoders(ngl_model* m, void* packed, size_t bytes, void* stream);

/* ------------------------------------------------------------------ */
/* 2. SDF query (Sec. 3.2, Eq. 2; continuous LOD, Eq. 3)                  */
/* ------------------------------------------------------------------ */

/* For each point x_p (device x[3][P]) the voxel containing it is found at
 * every level l <= L' (L' = lod, or lod+1 when blending): cells are
 * half-open [lo, hi) per axis with x = +1 in the last cell, computed
 * exactly; points outside [-1,1]^3 have no voxel.  psi_l is the trilinear
 * interpolation of the voxel's 8 corner features (0 if the voxel is absent),
 * z_L = sum_{l<=L} psi_l, and sdf = f_{theta_L}([x, z_L]) (one hidden ReLU
 * layer, linear output).  With alpha > 0 (scalar) or alpha_pp (device [P],
 * nullable, values in [0,1)), sdf = (1-a) f_L + a f_{L+1} (needs
 * lod < num_lods).
 * Outputs (device): sdf[P]; valid[P] (nullable): 1 iff the level-L' voxel
 * exists; vox_out[L'][P] (nullable): voxel index per level, -1 if absent.
 * The decoder's first layer runs in FP32 when w_dtype is F32 and on the
 * BF16 matrix cores with FP32 accumulation when w_dtype is BF16: the BF16
 * weights are used as stored and every FP32 input (z, x, b1) enters as the
 * sum of two BF16 values (relative representation error 2^-16).
 * Errors: NGL_E_INVALID for lod outside 1..num_lods, alpha outside [0,1),
 * blending at lod == num_lods, or null required pointers. */
int ngl_query_sdf(const ngl_model* m, const float* x, int64_t P, int32_t lod, float alpha,
                  const float* alpha_pp, float* sdf, uint8_t* valid, int32_t* vox_out, void* stream);

/* Decoder only (Eq. 2's per-LOD MLP, Sec. 4.1): sdf[p] = b2 + w2 . ReLU(W1
 * [x_p, z_p] + b1) of decoder `lod` for inputs the caller already holds —
 * the query with the feature gather split off.  x: device [3][P] FP32
 * (required iff with_xyz, else ignored); z: device [P][feat_dim] rows,
 * z_dtype NGL_F32 or NGL_BF16, 16-byte aligned; sdf: device [P] FP32.  The
 * decoder form follows the model's weights as in ngl_query_sdf (BF16
 * weights: matrix cores, BF16 rows used as stored, FP32 rows split into two
 * BF16 parts; FP32: NGL_OPT_F32_DECODER).
 * Errors: NGL_E_INVALID for bad arguments, NGL_E_UNSUPPORTED for an
 * uncompiled feat_dim. */
int ngl_decode_sdf(const ngl_model* m, int32_t lod, const float* x, const void* z, int32_t z_dtype, int64_t P,
                   float* sdf, void* stream);

/* Surface normals by central differences (App. A.4: normals are obtained by
 * finite differences).  For each point x_p (device x[3][P]) the gradient
 * g_a = (f(x + h e_a) - f(x - h e_a)) / (2h) of f = the SDF of
 * ngl_query_sdf at LOD lod (+alpha) is evaluated with six queries and
 * normals[3][P] (device) receives g / |g| (0 if |g| = 0).  With status
 * non-null the points are the hit points of rays instead: x = o + t_hit d
 * for rays whose status is NGL_RAY_HIT (o, d: [3][P], t_hit, status: [P]);
 * other rays get the zero vector.  h > 0. */
int ngl_sdf_normals(const ngl_model* m, const float* x, const float* o, const float* d, const float* t_hit,
                    const uint8_t* status, int64_t P, int32_t lod, float alpha, float h, float* normals,
                    void* stream);

/* All discrete LODs at once: sdf_all[L][P] (device) with sdf_all[L-1][p] =
 * f_{theta_L}([x_p, z_L(x_p)]) for L = 1..num_lods (the forward of Eq. 4). */
int ngl_query_sdf_all_lods(const ngl_model* m, const float* x, int64_t P, float* sdf_all, void* stream);

/* ------------------------------------------------------------------ */
/* 3. Rays: camera, ray-octree intersection (Sec. 3.4, Alg. 1, App. C),  */
/*    adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3, App. A.4)      */
/* ------------------------------------------------------------------ */

/* Pinhole primary rays of a width x height image (ray i = row*width+col,
 * row 0 at the top) through pixel centres, vertical field of view fov_y
 * (degrees).  Basis f = normalize(target-eye), r = normalize(f x up),
 * u = r x f; dir = normalize(f + sx*tan(fov/2)*aspect*r + sy*tan(fov/2)*u),
 * sx = 2(col+0.5)/width - 1, sy = 1 - 2(row+0.5)/height.
 * eye/target/up: host float[3]; o, d: device float[3][width*height]. */
int ngl_camera_rays(const float* eye, const float* target, const float* up, float fov_y_deg,
                    int32_t width, int32_t height, float* o, float* d, void* stream);

/* Bytes of device workspace needed by ngl_trace_octree for R rays and a
 * capacity of `pair_capacity` ray-voxel pairs per level. */
int ngl_trace_octree_workspace(int64_t R, int64_t pair_capacity, size_t* bytes);

/* Breadth-first ray-octree intersection (Alg. 1).  Starting from the pairs
 * (i, root) for every ray, each depth 0..target_depth runs Decide (FP32
 * slab test of the ray against the voxel's closed box; D = 1 at the target
 * depth, the number of occupied children otherwise, 0 on a miss),
 * ExclusiveSum of D, then Subdivide (children written front to back at the
 * exclusive-sum offset) or, at the target depth, Compactify.  Children are
 * ordered k = 0..7 as child k XOR oct, oct_a = 1 iff o_a > centre_a of the
 * parent voxel; this is front-to-back order (App. C).
 * The slab test per axis: inv = 1/d (correctly rounded); if inv is
 * infinite the axis passes iff lo <= o <= hi; else t0 = (lo-o)*inv,
 * t1 = (hi-o)*inv, near/far by compare-and-select; tmin = max near,
 * tmax = min far; hit iff tmax >= max(tmin, 0).
 * Inputs (device): o, d [3][R].  Outputs (device, capacity pair_capacity):
 * pair_ray, pair_vox, t_in = max(tmin, 0), t_out = tmax, ordered by ray
 * then front to back; ray_off[R+1] (int32): ray i owns [ray_off[i],
 * ray_off[i+1]).  counts (device int64[2]): counts[0] = final pair count,
 * counts[1] = the largest pair list needed at any depth.  If counts[1] >
 * pair_capacity the outputs are incomplete; the call cannot know this
 * without synchronising, so the caller checks counts after the stream
 * completes and retries with pair_capacity >= counts[1].  Lists deeper than
 * the first overflowing depth are built from a truncated list, so after an
 * overflow counts[1] is a lower bound: repeat until counts[1] fits.  No
 * buffer is ever written beyond pair_capacity entries.
 * ws: device workspace of ngl_trace_octree_workspace bytes.  NGL_E_INVALID
 * if target_depth is outside 0..num_lods+1 or buffers are null. */
int ngl_trace_octree(const ngl_model* m, const float* o, const float* d, int64_t R,
                     int32_t target_depth, int64_t pair_capacity, void* ws, size_t ws_bytes,
                     int32_t* pair_ray, int32_t* pair_vox, float* t_in, float* t_out,
                     int32_t* ray_off, int64_t* counts, void* stream);

typedef struct {
  int32_t max_steps;  /* SDF evaluations per ray (App. A.4 uses 200) */
  float delta;        /* hit threshold: stop when sdf < delta (App. A.4: 3e-4) */
  float t_far;        /* far-plane clip distance (App. A.4: 5) */
  int32_t osc_check;  /* 1: stop (STALLED) when |d_k - d_{k-1}| < 6 delta */
  int32_t analytic;   /* 1: replace the model by the exact SDF of `sphere` */
  float sphere[4];    /* cx, cy, cz, radius for analytic mode */
  int32_t image_width; /* > 0: the rays are an image of this width, row-major
                          (a multiple of 8, and R a multiple of 8 widths); they
                          are then handed to the wavefronts in 8x8 pixel tiles,
                          so a wavefront's rays meet nearby voxels.  0: in ray
                          order.  Results do not depend on it. */
} ngl_trace_params;

/* Adaptive-stepping sphere trace (Sec. 3.4, Fig. 3) over the hit lists of
 * ngl_trace_octree at depth L'+1 (L' = lod, or lod+1 if alpha > 0).  Per
 * ray, with cursor p over its pairs and t starting at the first t_in:
 * skip pairs whose t_out < t (empty space: next voxel; none left: MISS);
 * if t < t_in[p] advance t to it; t > t_far: FAR; step budget spent:
 * MAX_STEPS; otherwise evaluate the SDF at o + t d from voxel pair_vox[p]
 * and its ancestors (local coordinates clamped to the voxel), and stop
 * with HIT when it is below delta, else t += sdf.  t accumulates in FP32.
 * Outputs (device, [R]): t_hit (t at termination), status (ngl_ray_status),
 * steps (SDF evaluations), hit_vox (pair voxel at HIT, else -1).
 * The hit lists must come from ngl_trace_octree at depth L'+1 with the same
 * rays; a voxel index outside that depth ends its ray as INVALID.  Rays are
 * processed by a persistent grid whose lanes take the next ray from a queue
 * in `ws` when theirs ends; results do not depend on the schedule. */
int ngl_sphere_trace(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t lod,
                     float alpha, const int32_t* pair_vox, const float* t_in, const float* t_out,
                     const int32_t* ray_off, const ngl_trace_params* params, float* t_hit,
                     uint8_t* status, int32_t* steps, int32_t* hit_vox, void* ws, size_t ws_bytes,
                     void* stream);

/* Bytes of device workspace ngl_sphere_trace needs (a work-queue counter,
 * cleared by the call itself).  Calls that share a workspace must not run
 * concurrently. */
int ngl_sphere_trace_workspace(size_t* bytes);
/* Workspace that lets ngl_sphere_trace run in phases (about 24*R + 256
 * bytes): rays still running after NGL_OPT_TRACE_PAUSE1 (then
 * NGL_OPT_TRACE_PAUSE2) evaluations are parked with their state and served
 * again by the next launch from a dense queue, so the long grazing rays do
 * not keep near-empty wavefronts busy.  Results are the same bits as the
 * single launch (every ray takes the same steps from the same state).  A
 * workspace below this size runs the single launch. */
int ngl_sphere_trace_workspace_rays(int64_t R, size_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ngl_sphere_trace with its phased workspace in a device array the library
 * owns (one per GPU, NGL_STATIC_TRACE_BYTES, held until the process ends)
 * instead of a caller workspace.  Same arguments and results as
 * ngl_sphere_trace with a workspace of ngl_sphere_trace_workspace_rays(R)
 * bytes, for R <= NGL_STATIC_TRACE_MAX_RAYS (NGL_E_CAPACITY above).  The
 * call allocates nothing: it runs no hipMalloc/hipFree and the array's
 * counters are cleared by a kernel on `stream`.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams,
 * other threads) race: serialise them. */
#define NGL_STATIC_TRACE_MAX_RAYS (1 << 21)
#define NGL_STATIC_TRACE_BYTES (256 + 6 * 4 * (size_t)NGL_STATIC_TRACE_MAX_RAYS)
int ngl_sphere_trace_static(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t lod,
                            float alpha, const int32_t* pair_vox, const float* t_in, const float* t_out,
                            const int32_t* ray_off, const ngl_trace_params* params, float* t_hit,
                            uint8_t* status, int32_t* steps, int32_t* hit_vox, void* stream);

/* Per-pixel LOD selection (Sec. 3.4, LOD Selection): the continuous LOD of
 * a ray moves linearly from lod_near at distance d_near to lod_far at
 * d_far (constant outside), where the distance is the entry t of the ray's
 * first hit pair (params->t_far for a ray without pairs).  Evaluated in
 * FP32, each operation rounded in this order:
 *   u = clamp((dist - d_near) / (d_far - d_near), 0, 1)
 *   L = lod_near + (lod_far - lod_near) * u, clamped to [min, max] of the
 *       two LODs
 *   L* = floor(L), alpha = L - L*; L* = num_lods, alpha = 0 if L >= num_lods. */
typedef struct {
  float d_near, d_far;     /* d_far > d_near */
  float lod_near, lod_far; /* continuous LODs in [1, num_lods] */
} ngl_lod_select;

/* Sphere trace in which each ray uses its own LOD L* + alpha (Eq. 3) from
 * the heuristic above.  The hit lists (ngl_trace_octree output) are at
 * pair_depth, which must reach every selected level:
 * pair_depth - 1 >= ceil(max(lod_near, lod_far)), pair_depth <= num_lods+1;
 * each SDF evaluation of a ray uses the ancestors of its current pair's
 * voxel.  Rays are grouped by L* on the device and each group is traced by
 * one persistent launch with the decoders L* and L*+1.  Outputs as in
 * ngl_sphere_trace (hit_vox is a voxel at pair_depth), plus lod_out
 * (nullable, device [R]): each ray's continuous LOD L.  ws: device bytes
 * from ngl_sphere_trace_lod_workspace(R); calls sharing it must not
 * overlap.  With matrix-core decoders and that workspace the groups are
 * traced in two phases as in ngl_sphere_trace (rays still running after
 * NGL_OPT_TRACE_PAUSE1 evaluations are parked per group and finished with
 * a group of lanes per ray; same results bit for bit); a workspace of
 * 256 + 9 R bytes (rounded up per array) runs one phase. */
int ngl_sphere_trace_lod_workspace(int64_t R, size_t* bytes);
int ngl_sphere_trace_lod(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t pair_depth,
                         const ngl_lod_select* sel, const int32_t* pair_vox, const float* t_in, const float* t_out,
                         const int32_t* ray_off, const ngl_trace_params* params, float* t_hit, uint8_t* status,
                         int32_t* steps, int32_t* hit_vox, float* lod_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* 3b. Batched rendering of several models (each its own octree, camera   */
/*     and LOD) with one persistent sphere-tracing launch.                */
/* ------------------------------------------------------------------ */
#define NGL_MAX_BATCH 32

typedef struct {
  float eye[3], target[3], up[3];  /* camera as in ngl_camera_rays */
  float fov_y_deg;
  int32_t width, height;
  int32_t lod;                     /* LOD traced (1..num_lods of the view's model) */
  float alpha;                     /* continuous LOD lod + alpha, in [0,1) */
} ngl_view;

/* Device copy of up to NGL_MAX_BATCH model views for the batched tracer.
 * ngl_model_table_upload copies the host array into `table` (device, at
 * least ngl_model_table_bytes bytes) and synchronises `stream`, so the host
 * array may be released on return.  Re-upload when a model changes. */
int ngl_model_table_bytes(int32_t n, size_t* bytes);
int ngl_model_table_upload(const ngl_model* models, int32_t n, void* table, void* stream);

/* Workspace bytes of ngl_render_batch for these views and a per-view pair
 * capacity (see ngl_trace_octree). */
int ngl_render_batch_workspace(const ngl_view* views, int32_t n, int64_t pair_capacity, size_t* bytes);

/* Renders view i of model i (i < n <= NGL_MAX_BATCH): camera rays, the
 * ray-octree intersection at the depth of LOD lod (lod+1 if alpha > 0),
 * then ONE persistent sphere-trace launch for all views: each block takes
 * a view, stages that model's decoder in LDS and serves the view's ray
 * queue with lane refill (every step runs on compacted active rays), then
 * moves on to views with work left.  All models must share feat_dim,
 * hidden, with_xyz, feat_dtype and w_dtype.  models: host array (checked);
 * table: its device copy from ngl_model_table_upload.  Outputs (device)
 * concatenate the views in order, view i owning width*height entries:
 * t_hit, status, steps, hit_vox as in ngl_sphere_trace.  counts (device
 * int64 [n][2]) as in ngl_trace_octree per view; if any counts[i][1] >
 * pair_capacity the render is incomplete (retry with a larger capacity).
 * frame_clock (device uint64 [n+1], nullable): [0] a device wall-clock
 * timestamp (100 MHz) taken when the batch starts, [i+1] when view i's last
 * ray ends.  No host synchronisation; safe to capture in a graph. */
int ngl_render_batch(const ngl_model* models, const void* table, const ngl_view* views, int32_t n,
                     const ngl_trace_params* params, int64_t pair_capacity, void* ws, size_t ws_bytes,
                     float* t_hit, uint8_t* status, int32_t* steps, int32_t* hit_vox, int64_t* counts,
                     uint64_t* frame_clock, void* stream);

/* ------------------------------------------------------------------ */
/* 4. Training (Sec. 3.3, Eq. 4)                                        */
/* ------------------------------------------------------------------ */

/* Bytes of device workspace for the backward / training step on P points. */
int ngl_train_workspace(const ngl_model* m, int64_t P, size_t* bytes);

/* Gradient of sum_{L,p} grad_sdf[L-1][p] * sdf_all[L-1][p] with respect to
 * every parameter, given the upstream gradient grad_sdf (device [L][P]).
 * Feature gradients are accumulated without atomics (points are sorted by
 * voxel, then each corner gathers its contributions in a fixed order), so
 * results are bitwise reproducible.  Outputs (device, float32, overwritten):
 * dfeat[l] [ncorner][m], dW1[l] [h][din], db1[l] [h], dw2[l] [h], db2 [L].
 * Requires feat_dtype == F32 and w_dtype == F32. */
int ngl_backward_all_lods(const ngl_model* m, const float* x, int64_t P, const float* grad_sdf,
                          float* const* dfeat, float* const* dW1, float* const* db1,
                          float* const* dw2, float* db2, void* ws, size_t ws_bytes, void* stream);

/* One training forward+backward of Eq. 4: loss = (1/P) sum_p sum_L
 * (sdf_L(x_p) - target_p)^2 written to loss (device float[1]), sdf_all
 * (device [L][P], nullable) and gradients as in ngl_backward_all_lods. */
int ngl_train_fwd_bwd(const ngl_model* m, const float* x, const float* target, int64_t P,
                      float* loss, float* sdf_all, float* const* dfeat, float* const* dW1,
                      float* const* db1, float* const* dw2, float* db2, void* ws,
                      size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* 5. Fitting (training appendix): analytic shapes, samplers, Adam        */
/* ------------------------------------------------------------------ */
/* Synthetic ground-truth shape: union of spheres [cx, cy, cz, R] and tori
 * [cx, cy, cz, R, r, axis] (axis 0/1/2 = x/y/z; the ring lies in the plane
 * of the other two coordinates), FP32 device arrays.  Its SDF is the
 * minimum of the primitives' exact signed distances. */
typedef struct {
  int32_t n_spheres, n_tori;
  const float* spheres; /* device [n_spheres][4] */
  const float* tori;    /* device [n_tori][6] */
} ngl_shape;

/* sdf[p] = union SDF at x[.][p] (device [3][P] in, device [P] out). */
int ngl_shape_sdf(const ngl_shape* shape, const float* x, int64_t P, float* sdf, void* stream);

/* SDF surface sampler (training appendix, Sampling): candidate ray i starts
 * at -1 + 2 (u0, u1, u2) with direction (sqrt(1-z^2) cos phi,
 * sqrt(1-z^2) sin phi, z), z = 1 - 2 u3, phi = 2 pi u4 (u: device [5][n]
 * uniforms in [0, 1]); it takes |SDF| steps from t = 0 and hits when
 * |SDF| < delta, misses on leaving [-1, 1]^3 or after max_steps.  The hit
 * points are written compacted in ray order to pts (device [3][n], stride
 * n) and their number to *count (device int64).  ws: device bytes from
 * ngl_sample_surface_workspace(n). */
int ngl_sample_surface_workspace(int64_t n, size_t* bytes);
int ngl_sample_surface(const ngl_shape* shape, const float* u, int64_t n, int32_t max_steps, float delta,
                       float* pts, int64_t* count, void* ws, size_t ws_bytes, void* stream);

/* Training set of N points (training appendix: 2:2:1 surface, near,
 * uniform), interleaved so that point i (q = i / 5, c = i % 5) is surface
 * sample S[2q + c] (c = 0, 1), S[2q + c - 2] plus sigma times a standard
 * normal triple from Box-Muller on (u0, u1), (u2, u3) (c = 2, 3; a radius
 * input of 0 reads as 1), or -1 + 2 (u0, u1, u2) (c = 4), with u = uniforms
 * [.][i] (device [4][N]) and the n_surface samples S (device [3][stride])
 * used cyclically.  x is written batch-major, device [N/batch][3][batch]
 * (N a multiple of batch), target[i] (device [N]) = the shape's SDF at
 * point i. */
int ngl_training_points(const ngl_shape* shape, const float* surface, int64_t n_surface, int64_t surface_stride,
                        const float* uniforms, int64_t N, int64_t batch, float sigma, float* x, float* target,
                        void* stream);

/* One Adam step (Kingma and Ba 2015, Algorithm 1) over n <= 64 FP32 device
 * tensors in one launch: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m c1) / (sqrt(v c2) + eps), c1 = 1/(1 - b1^step),
 * c2 = 1/(1 - b2^step) (host FP64, rounded to FP32).  param/grad/m/v: host
 * arrays of n device pointers, numel: host [n].  step >= 1. */
#define NGL_MAX_ADAM_TENSORS 64
typedef struct {
  float lr, beta1, beta2, eps;
  int32_t step;
} ngl_adam_params;
int ngl_adam_step(const ngl_adam_params* p, int32_t n, float* const* param, const float* const* grad,
                  float* const* m, float* const* v, const int64_t* numel, void* stream);

/* Eq. 4 with a weight per LOD (host [num_lods], finite, >= 0):
 * J = (1/P) sum_p sum_L w_L (dhat_L - d)^2.  Weight 0 removes a LOD's
 * term (progressive schedule of the training appendix); all ones is
 * ngl_train_fwd_bwd. */
int ngl_train_fwd_bwd_lods(const ngl_model* m, const float* x, const float* target, int64_t P,
                           const float* lod_weight, float* loss, float* sdf_all, float* const* dfeat,
                           float* const* dW1, float* const* db1, float* const* dw2, float* db2, void* ws,
                           size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* 6. Workspace sizes in one call                                        */
/* ------------------------------------------------------------------ */
typedef enum {
  NGL_OP_TRACE_OCTREE = 0,        /* n = rays, aux = pair capacity per depth */
  NGL_OP_SPHERE_TRACE = 1,        /* n = rays: the phased trace's workspace */
  NGL_OP_SPHERE_TRACE_LOD = 2,    /* n = rays */
  NGL_OP_TRAIN = 3,               /* n = points; needs the model */
  NGL_OP_SAMPLE_SURFACE = 4,      /* n = candidate rays */
  NGL_OP_OCTREE_BUILD_DEVICE = 5, /* n = occupied cells, aux = num_lods */
  NGL_OP_PACK_DECODERS = 6        /* bytes of ngl_pack_decoders; needs the model */
} ngl_op;

/* Device bytes the call `op` needs for n items: the same value as that
 * call's own size query (ngl_trace_octree_workspace,
 * ngl_sphere_trace_workspace_rays, ngl_sphere_trace_lod_workspace,
 * ngl_train_workspace, ngl_sample_surface_workspace,
 * ngl_octree_build_device_workspace, ngl_packed_decoder_bytes), so a caller
 * can size every buffer through one entry point.  m may be NULL except for
 * NGL_OP_TRAIN and NGL_OP_PACK_DECODERS.  The batched render's workspace
 * depends on its views and has its own query (ngl_render_batch_workspace).
 * NGL_E_INVALID for an unknown op, negative sizes or a missing model. */
int ngl_workspace_bytes(int op, const ngl_model* m, int64_t n, int64_t aux, size_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* NGL_H */
