/*
 * FP64 CPU oracle for the neural geometric LOD hot path (Takikawa et al.,
 * "Neural Geometric Level of Detail", arXiv 2101.10994).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a deliberately plain, slow and
 * obviously correct restatement of what the paper computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the GPU library never links, includes or calls it, and it includes
 * nothing from the GPU library.
 *
 * Data structures are sorted arrays of Morton codes searched with bsearch:
 * a voxel's canonical index at a depth is the rank of its Morton code among
 * that depth's voxels, a corner's canonical index at a feature level is the
 * rank of its lattice Morton code.  Every lookup below is that definition.
 *
 * Conventions (the paper fixes none of these orders; see the design notes):
 *   - feature level l (1-based) has grid resolution r_l = 4 * 2^(l-1) and
 *     lives at octree depth l+1; depth d has resolution 2^d (App. A.1);
 *   - Morton code: bit 3k+0 = x, 3k+1 = y, 3k+2 = z, coarser bits higher;
 *   - child index c = cx | cy<<1 | cz<<2, corner slot j = a | b<<1 | c<<2.
 *
 * Precision: FP64 everywhere except the ray/box slab predicate, which is
 * specified in FP32 so that hit lists can be compared bit for bit.  Build
 * with -ffp-contract=off and without fast-math.
 *
 * Parity status of each entry point is listed in the oracle's Python
 * wrapper; all are pinned by tests that do not reuse this code.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXL 10             /* feature levels */
#define ORC_MAXD (ORC_MAXL + 2) /* depths 0..MAXL+1 */

/* ------------------------------------------------------------------ */
/* Morton codes                                                        */
/* ------------------------------------------------------------------ */
static uint64_t morton3(uint64_t x, uint64_t y, uint64_t z) {
  uint64_t code = 0;
  for (int b = 0; b < 20; ++b) {
    code |= ((x >> b) & 1ull) << (3 * b + 0);
    code |= ((y >> b) & 1ull) << (3 * b + 1);
    code |= ((z >> b) & 1ull) << (3 * b + 2);
  }
  return code;
}

static void demorton3(uint64_t code, int64_t* x, int64_t* y, int64_t* z) {
  *x = *y = *z = 0;
  for (int b = 0; b < 20; ++b) {
    *x |= (int64_t)((code >> (3 * b + 0)) & 1ull) << b;
    *y |= (int64_t)((code >> (3 * b + 1)) & 1ull) << b;
    *z |= (int64_t)((code >> (3 * b + 2)) & 1ull) << b;
  }
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/* Sort and drop duplicates; returns the new length. */
static int64_t sort_unique(uint64_t* v, int64_t n) {
  if (n == 0) return 0;
  qsort(v, (size_t)n, sizeof(uint64_t), cmp_u64);
  int64_t k = 1;
  for (int64_t i = 1; i < n; ++i)
    if (v[i] != v[k - 1]) v[k++] = v[i];
  return k;
}

/* Rank of `key` in sorted array v[0..n), or -1 if absent. */
static int64_t rank_of(const uint64_t* v, int64_t n, uint64_t key) {
  const uint64_t* p = (const uint64_t*)bsearch(&key, v, (size_t)n, sizeof(uint64_t), cmp_u64);
  return p ? (int64_t)(p - v) : -1;
}

/* ------------------------------------------------------------------ */
/* Octree (Sec. 3.2: voxels exist only where there is surface; parents  */
/* always exist, Sec. 3.4)                                               */
/* ------------------------------------------------------------------ */
typedef struct {
  int num_lods;                     /* Lmax */
  int depth;                        /* D = Lmax + 1 (finest depth) */
  int64_t nvox[ORC_MAXD];           /* voxels per depth 0..D */
  uint64_t* code[ORC_MAXD];         /* sorted voxel Morton codes per depth */
  int64_t ncorner[ORC_MAXL];        /* corners per feature level 1..Lmax */
  uint64_t* corner_code[ORC_MAXL];  /* sorted lattice Morton codes */
} orc_octree;

void orc_octree_free(orc_octree* t) {
  if (!t) return;
  for (int d = 0; d < ORC_MAXD; ++d) free(t->code[d]);
  for (int l = 0; l < ORC_MAXL; ++l) free(t->corner_code[l]);
  free(t);
}

/*
 * Build from finest-level occupied cells ijk[n][3] at resolution 2^(Lmax+1).
 * Depth-d voxels are the parent closure {cell >> (D-d)}; feature level l's
 * corners are the union of the 8 lattice points of its voxels.
 * Returns NULL on invalid input.
 */
orc_octree* orc_octree_build(const int32_t* ijk, int64_t n, int num_lods) {
  if (num_lods < 1 || num_lods > ORC_MAXL || n < 0) return NULL;
  orc_octree* t = (orc_octree*)calloc(1, sizeof(orc_octree));
  t->num_lods = num_lods;
  t->depth = num_lods + 1;
  const int D = t->depth;
  const int64_t res = (int64_t)1 << D;
  for (int64_t k = 0; k < n; ++k)
    for (int a = 0; a < 3; ++a)
      if (ijk[3 * k + a] < 0 || ijk[3 * k + a] >= res) { orc_octree_free(t); return NULL; }
  for (int d = 0; d <= D; ++d) {
    uint64_t* v = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int s = D - d;
    for (int64_t k = 0; k < n; ++k)
      v[k] = morton3((uint64_t)(ijk[3 * k] >> s), (uint64_t)(ijk[3 * k + 1] >> s),
                     (uint64_t)(ijk[3 * k + 2] >> s));
    t->nvox[d] = sort_unique(v, n);
    t->code[d] = v;
  }
  for (int l = 1; l <= num_lods; ++l) {
    int d = l + 1;
    int64_t nv = t->nvox[d];
    uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(8 * nv > 0 ? 8 * nv : 1));
    for (int64_t v = 0; v < nv; ++v) {
      int64_t x, y, z;
      demorton3(t->code[d][v], &x, &y, &z);
      for (int j = 0; j < 8; ++j)
        c[8 * v + j] = morton3((uint64_t)(x + (j & 1)), (uint64_t)(y + ((j >> 1) & 1)),
                               (uint64_t)(z + ((j >> 2) & 1)));
    }
    t->ncorner[l - 1] = sort_unique(c, 8 * nv);
    t->corner_code[l - 1] = c;
  }
  return t;
}

void orc_octree_counts(const orc_octree* t, int64_t* nvox, int64_t* ncorner) {
  for (int d = 0; d <= t->depth; ++d) nvox[d] = t->nvox[d];
  for (int l = 0; l < t->num_lods; ++l) ncorner[l] = t->ncorner[l];
}

/* Voxel index at `depth` of cell (x,y,z), or -1. */
static int64_t voxel_index(const orc_octree* t, int depth, int64_t x, int64_t y, int64_t z) {
  int64_t r = (int64_t)1 << depth;
  if (x < 0 || y < 0 || z < 0 || x >= r || y >= r || z >= r) return -1;
  return rank_of(t->code[depth], t->nvox[depth], morton3((uint64_t)x, (uint64_t)y, (uint64_t)z));
}

/* Corner index at feature level l of lattice point (x,y,z), or -1. */
static int64_t corner_index(const orc_octree* t, int l, int64_t x, int64_t y, int64_t z) {
  return rank_of(t->corner_code[l - 1], t->ncorner[l - 1], morton3((uint64_t)x, (uint64_t)y, (uint64_t)z));
}

/*
 * Export the per-depth structure arrays in the canonical layout, each
 * computed from its definition:
 *   ijk[v][3]       cell of voxel v,
 *   child_mask[v]   bit c set iff child c exists (d < D),
 *   first_child[v]  index of the lowest existing child at depth d+1, or -1,
 *   parent[v]       index of the parent at depth d-1 (-1 at the root).
 */
void orc_octree_export_depth(const orc_octree* t, int d, int32_t* ijk, uint8_t* child_mask,
                             int32_t* first_child, int32_t* parent) {
  for (int64_t v = 0; v < t->nvox[d]; ++v) {
    int64_t x, y, z;
    demorton3(t->code[d][v], &x, &y, &z);
    if (ijk) { ijk[3 * v] = (int32_t)x; ijk[3 * v + 1] = (int32_t)y; ijk[3 * v + 2] = (int32_t)z; }
    if (child_mask || first_child) {
      uint8_t mask = 0;
      int64_t first = -1;
      if (d < t->depth) {
        for (int c = 0; c < 8; ++c) {
          int64_t ci = voxel_index(t, d + 1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1));
          if (ci >= 0) {
            mask |= (uint8_t)(1u << c);
            if (first < 0 || ci < first) first = ci;
          }
        }
      }
      if (child_mask) child_mask[v] = mask;
      if (first_child) first_child[v] = (int32_t)first;
    }
    if (parent) parent[v] = d == 0 ? -1 : (int32_t)voxel_index(t, d - 1, x >> 1, y >> 1, z >> 1);
  }
}

/* Corner table of feature level l: corners[v][j] for the voxels at depth l+1,
 * and the lattice coordinates of each corner (corner_ijk[c][3]). */
void orc_octree_export_corners(const orc_octree* t, int l, int32_t* corners, int32_t* corner_ijk) {
  int d = l + 1;
  if (corners) {
    for (int64_t v = 0; v < t->nvox[d]; ++v) {
      int64_t x, y, z;
      demorton3(t->code[d][v], &x, &y, &z);
      for (int j = 0; j < 8; ++j)
        corners[8 * v + j] = (int32_t)corner_index(t, l, x + (j & 1), y + ((j >> 1) & 1), z + ((j >> 2) & 1));
    }
  }
  if (corner_ijk) {
    for (int64_t c = 0; c < t->ncorner[l - 1]; ++c) {
      int64_t x, y, z;
      demorton3(t->corner_code[l - 1][c], &x, &y, &z);
      corner_ijk[3 * c] = (int32_t)x; corner_ijk[3 * c + 1] = (int32_t)y; corner_ijk[3 * c + 2] = (int32_t)z;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Model: corner features and per-LOD decoders (Sec. 3.2, Eq. 2)        */
/* ------------------------------------------------------------------ */
typedef struct {
  int num_lods;                 /* Lmax */
  int m;                        /* feature dim */
  int hidden;                   /* decoder hidden width */
  int with_xyz;                 /* decoder input [x, z] (1) or [z] (0) */
  const double* feat[ORC_MAXL]; /* [ncorner_l][m] */
  const double* W1[ORC_MAXL];   /* [hidden][din] */
  const double* b1[ORC_MAXL];   /* [hidden] */
  const double* w2[ORC_MAXL];   /* [hidden] */
  const double* b2;             /* [Lmax] */
} orc_model;

static int din_of(const orc_model* M) { return M->m + (M->with_xyz ? 3 : 0); }

/* Half-open cell [lo, hi) of resolution r containing x in [-1, 1]; x = +1
 * belongs to the last cell.  Exact: the floating estimate is corrected by
 * comparisons against the exact dyadic cell bounds. */
static int64_t cell_of(double x, int64_t r) {
  double f = floor((x + 1.0) * (double)r * 0.5);
  int64_t i = (int64_t)f;
  if (i < 0) i = 0;
  if (i > r - 1) i = r - 1;
  while (i > 0 && x < -1.0 + 2.0 * (double)i / (double)r) --i;
  while (i < r - 1 && x >= -1.0 + 2.0 * (double)(i + 1) / (double)r) ++i;
  return i;
}

static int in_box(const double x[3]) {
  for (int a = 0; a < 3; ++a)
    if (!(x[a] >= -1.0 && x[a] <= 1.0)) return 0; /* also rejects NaN */
  return 1;
}

/* psi(x; l) for cell (ix,iy,iz) of level l: trilinear interpolation of the
 * 8 corner features (Sec. 3.2).  u is the position inside the cell, clamped
 * to [0,1]. */
static void interp_level(const orc_octree* t, const orc_model* M, int l, const int64_t cell[3],
                         const double x[3], double* psi /* [m] */) {
  int64_t r = (int64_t)1 << (l + 1);
  double u[3];
  for (int a = 0; a < 3; ++a) {
    double lo = -1.0 + 2.0 * (double)cell[a] / (double)r;
    u[a] = (x[a] - lo) * (double)r / 2.0;
    if (u[a] < 0.0) u[a] = 0.0;
    if (u[a] > 1.0) u[a] = 1.0;
  }
  for (int k = 0; k < M->m; ++k) psi[k] = 0.0;
  for (int j = 0; j < 8; ++j) {
    int b[3] = {j & 1, (j >> 1) & 1, (j >> 2) & 1};
    double w = 1.0;
    for (int a = 0; a < 3; ++a) w *= b[a] ? u[a] : 1.0 - u[a];
    int64_t c = corner_index(t, l, cell[0] + b[0], cell[1] + b[1], cell[2] + b[2]);
    const double* z = M->feat[l - 1] + (size_t)c * (size_t)M->m;
    for (int k = 0; k < M->m; ++k) psi[k] += w * z[k];
  }
}

/* One decoder f_{theta_L}([x, z]) (Eq. 2): linear -> ReLU -> linear.
 * Also returns two magnitude scales for error bounds (not part of the
 * method): scale = |b2| + sum_k |w2_k h_k| (cancellation in the last dot
 * product) and scale1 = |b2| + sum_k |w2_k| (|b1_k| + sum_i |W1_ki in_i|)
 * (magnitude of the first layer's products, which bounds the effect of
 * rounding the first layer's inputs). */
static double decode(const orc_model* M, int L, const double x[3], const double* z, double* scale,
                     double* scale1) {
  int din = din_of(M), H = M->hidden;
  const double* W1 = M->W1[L - 1];
  const double* b1 = M->b1[L - 1];
  const double* w2 = M->w2[L - 1];
  double out = M->b2[L - 1];
  double s = fabs(M->b2[L - 1]);
  double s1 = fabs(M->b2[L - 1]);
  for (int k = 0; k < H; ++k) {
    double a = b1[k];
    double mag = fabs(b1[k]);
    int col = 0;
    if (M->with_xyz)
      for (int q = 0; q < 3; ++q) {
        a += W1[(size_t)k * din + col] * x[q];
        mag += fabs(W1[(size_t)k * din + col] * x[q]);
        ++col;
      }
    for (int q = 0; q < M->m; ++q) {
      a += W1[(size_t)k * din + col] * z[q];
      mag += fabs(W1[(size_t)k * din + col] * z[q]);
      ++col;
    }
    double h = a > 0.0 ? a : 0.0;
    out += w2[k] * h;
    s += fabs(w2[k] * h);
    s1 += fabs(w2[k]) * mag;
  }
  if (scale) *scale = s;
  if (scale1) *scale1 = s1;
  return out;
}

/*
 * Decoder only (Eq. 2's MLP of LOD `lod`) on given inputs: x SoA [3][P]
 * float (ignored without the position input), z [P][m] double rows.
 * Outputs sdf[P] and the two magnitude scales of decode (nullable).
 * Returns 0, or -1 on invalid arguments.
 */
int orc_decode(const orc_model* M, int lod, const float* xs, const double* zs, int64_t P, double* sdf,
               double* scale, double* scale1) {
  if (lod < 1 || lod > M->num_lods) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < P; ++p) {
    double x[3] = {0.0, 0.0, 0.0};
    if (M->with_xyz)
      for (int a = 0; a < 3; ++a) x[a] = xs[(size_t)a * (size_t)P + (size_t)p];
    double s0, s1;
    sdf[p] = decode(M, lod, x, zs + (size_t)p * (size_t)M->m, &s0, &s1);
    if (scale) scale[p] = s0;
    if (scale1) scale1[p] = s1;
  }
  return 0;
}

/*
 * SDF query (Sec. 3.2 Eq. 2, blended per Eq. 3).
 *   x: SoA [3][P] float; lod in 1..Lmax; alpha in [0,1) applies to all points
 *   unless alpha_pp (nullable, [P]) is given.  alpha > 0 needs lod < Lmax.
 * For every level l <= L' (L' = lod, or lod+1 when blending), the voxel of
 * depth l+1 containing x is looked up; a missing voxel contributes psi = 0.
 * Outputs sdf[P], scale[P] and scale1[P] (the magnitude scales of decode,
 * blended like the sdf; nullable), valid[P] (voxel at level L' exists) and, if
 * vox_out is not NULL, vox_out[l-1][P] for l = 1..L' (-1 when absent).
 * Returns 0, or -1 on invalid arguments.
 */
int orc_query(const orc_octree* t, const orc_model* M, const float* xs, int64_t P, int lod,
              double alpha, const float* alpha_pp, double* sdf, double* scale, double* scale1, uint8_t* valid,
              int32_t* vox_out) {
  if (lod < 1 || lod > M->num_lods || M->num_lods != t->num_lods) return -1;
  int need_next = alpha_pp != NULL || alpha > 0.0;
  if (need_next && lod >= M->num_lods) return -1;
  int Lp = need_next ? lod + 1 : lod;
  int m = M->m;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < P; ++p) {
    double x[3] = {xs[p], xs[P + p], xs[2 * P + p]};
    double a = alpha_pp ? (double)alpha_pp[p] : alpha;
    double* z = (double*)calloc((size_t)m, sizeof(double));
    double* psi = (double*)calloc((size_t)m, sizeof(double));
    double* z_next = (double*)calloc((size_t)m, sizeof(double));
    int ok = in_box(x);
    int last_exists = 0;
    for (int l = 1; l <= Lp; ++l) {
      int64_t r = (int64_t)1 << (l + 1);
      int64_t cell[3] = {0, 0, 0};
      int64_t v = -1;
      if (ok) {
        for (int q = 0; q < 3; ++q) cell[q] = cell_of(x[q], r);
        v = voxel_index(t, l + 1, cell[0], cell[1], cell[2]);
      }
      if (vox_out) vox_out[(size_t)(l - 1) * (size_t)P + (size_t)p] = (int32_t)v;
      if (v >= 0) interp_level(t, M, l, cell, x, psi);
      else for (int k = 0; k < m; ++k) psi[k] = 0.0;
      if (l <= lod) for (int k = 0; k < m; ++k) z[k] += psi[k];
      else for (int k = 0; k < m; ++k) z_next[k] = z[k] + psi[k];
      if (l == Lp) last_exists = v >= 0;
    }
    double s0, s1 = 0.0, r0, r1 = 0.0;
    double d0 = decode(M, lod, x, z, &s0, &r0);
    double d = d0, s = s0, r = r0;
    if (need_next) {
      double d1 = decode(M, lod + 1, x, z_next, &s1, &r1);
      d = (1.0 - a) * d0 + a * d1;
      s = (1.0 - a) * s0 + a * s1;
      r = (1.0 - a) * r0 + a * r1;
    }
    sdf[p] = d;
    if (scale) scale[p] = s;
    if (scale1) scale1[p] = r;
    if (valid) valid[p] = (uint8_t)last_exists;
    free(z); free(psi); free(z_next);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Ray / box slab predicate, FP32 (the oracle's only FP32 code)          */
/* ------------------------------------------------------------------ */
/*
 * Box [lo, hi] (closed) given by exact dyadic bounds.  For each axis:
 *   inv = 1/d (correctly rounded); if inv is infinite the axis passes iff
 *   lo <= o <= hi; otherwise t0 = (lo-o)*inv, t1 = (hi-o)*inv (each op
 *   rounded separately), near = smaller, far = larger.
 * tmin = max(near over axes, starting at -inf), tmax = min(far, from +inf),
 * both by compare-and-select.  hit iff tmax >= max(tmin, 0);
 * t_in = tmin if tmin > 0 else 0, t_out = tmax.
 */
static int slab_f32(const float o[3], const float inv[3], const float lo[3], const float hi[3],
                    float* t_in, float* t_out) {
  float tmin = -INFINITY, tmax = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (isinf(inv[a])) {
      if (!(lo[a] <= o[a] && o[a] <= hi[a])) return 0;
      continue;
    }
    float d0 = lo[a] - o[a];
    float d1 = hi[a] - o[a];
    float t0 = d0 * inv[a];
    float t1 = d1 * inv[a];
    float nr = t0 < t1 ? t0 : t1;
    float fr = t0 < t1 ? t1 : t0;
    if (nr > tmin) tmin = nr;
    if (fr < tmax) tmax = fr;
  }
  float t0c = tmin > 0.0f ? tmin : 0.0f;
  if (!(tmax >= t0c)) return 0;
  *t_in = t0c;
  *t_out = tmax;
  return 1;
}

static void box_f32(int depth, const int64_t cell[3], float lo[3], float hi[3]) {
  int64_t r = (int64_t)1 << depth;
  for (int a = 0; a < 3; ++a) {
    lo[a] = (float)(-1.0 + 2.0 * (double)cell[a] / (double)r);
    hi[a] = (float)(-1.0 + 2.0 * (double)(cell[a] + 1) / (double)r);
  }
}

/* Exposed for tests: slab predicate of one ray against one cell. */
int orc_ray_box(const float o[3], const float d[3], int depth, const int32_t cell[3], float* t_in,
                float* t_out) {
  float inv[3], lo[3], hi[3];
  int64_t c[3] = {cell[0], cell[1], cell[2]};
  for (int a = 0; a < 3; ++a) inv[a] = 1.0f / d[a];
  box_f32(depth, c, lo, hi);
  return slab_f32(o, inv, lo, hi, t_in, t_out);
}

/* ------------------------------------------------------------------ */
/* Ray-octree intersection (Sec. 3.4, Alg. 1) as a per-ray depth-first */
/* search: from the root, a hit voxel either is emitted (target depth)   */
/* or has its occupied children visited front to back.  The children's   */
/* order depends only on which octant of the voxel holds the origin:     */
/* visiting k = 0..7 as child k XOR oct, oct_a = (o_a > centre_a).        */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int64_t cap;
  int32_t* vox;
  float* tin;
  float* tout;
} hitlist;

static void dfs(const orc_octree* t, int target, const float o[3], const float inv[3], int depth,
                const int64_t cell[3], hitlist* out) {
  float lo[3], hi[3], ti, to;
  box_f32(depth, cell, lo, hi);
  if (!slab_f32(o, inv, lo, hi, &ti, &to)) return;
  if (depth == target) {
    if (out->vox && out->n < out->cap) {
      out->vox[out->n] = (int32_t)voxel_index(t, depth, cell[0], cell[1], cell[2]);
      out->tin[out->n] = ti;
      out->tout[out->n] = to;
    }
    out->n++;
    return;
  }
  int64_t r = (int64_t)1 << depth;
  int oct = 0;
  for (int a = 0; a < 3; ++a) {
    /* centre = -1 + (2*cell+1)/r, exact */
    double centre = -1.0 + (2.0 * (double)cell[a] + 1.0) / (double)r;
    if ((double)o[a] > centre) oct |= 1 << a;
  }
  for (int k = 0; k < 8; ++k) {
    int c = k ^ oct;
    int64_t child[3] = {2 * cell[0] + (c & 1), 2 * cell[1] + ((c >> 1) & 1), 2 * cell[2] + ((c >> 2) & 1)};
    if (voxel_index(t, depth + 1, child[0], child[1], child[2]) >= 0) dfs(t, target, o, inv, depth + 1, child, out);
  }
}

/*
 * Hit lists of R rays (o, d: SoA [3][R] float) at octree depth `target`
 * (0..D).  Output, ordered by ray and front to back within a ray:
 * pair_ray/pair_vox/t_in/t_out [count], ray_off[R+1].  If the total exceeds
 * `capacity` nothing is written beyond ray_off and the total is returned.
 * Returns the total number of pairs, or -1 on invalid arguments.
 */
int64_t orc_trace_octree(const orc_octree* t, const float* o, const float* d, int64_t R, int target,
                         int64_t capacity, int32_t* pair_ray, int32_t* pair_vox, float* t_in,
                         float* t_out, int64_t* ray_off) {
  if (target < 0 || target > t->depth) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)R + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < R; ++i) {
    float oo[3] = {o[i], o[R + i], o[2 * R + i]};
    float inv[3];
    for (int a = 0; a < 3; ++a) inv[a] = 1.0f / d[a * R + i];
    hitlist hl = {0, 0, NULL, NULL, NULL};
    int64_t root[3] = {0, 0, 0};
    if (t->nvox[0] > 0) dfs(t, target, oo, inv, 0, root, &hl);
    cnt[i] = hl.n;
  }
  int64_t total = 0;
  for (int64_t i = 0; i < R; ++i) {
    ray_off[i] = total;
    total += cnt[i];
  }
  ray_off[R] = total;
  if (total <= capacity) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < R; ++i) {
      float oo[3] = {o[i], o[R + i], o[2 * R + i]};
      float inv[3];
      for (int a = 0; a < 3; ++a) inv[a] = 1.0f / d[a * R + i];
      int64_t b = ray_off[i];
      hitlist hl = {0, cnt[i], pair_vox + b, t_in + b, t_out + b};
      int64_t root[3] = {0, 0, 0};
      if (t->nvox[0] > 0) dfs(t, target, oo, inv, 0, root, &hl);
      for (int64_t k = 0; k < cnt[i]; ++k) pair_ray[b + k] = (int32_t)i;
    }
  }
  free(cnt);
  return total;
}

/* ------------------------------------------------------------------ */
/* Pinhole camera rays                                                  */
/* ------------------------------------------------------------------ */
/*
 * Primary rays through pixel centres (i+0.5, j+0.5) of a W x H image,
 * vertical field of view fov_y (degrees), row 0 at the top.  Basis:
 * f = normalize(target - eye), r = normalize(f x up), u = r x f.
 * Ray i = row*W + col:  dir = normalize(f + sx*tan*aspect*r + sy*tan*u),
 * sx = 2(col+0.5)/W - 1, sy = 1 - 2(row+0.5)/H.  Output SoA [3][W*H].
 */
void orc_camera_rays(const double eye[3], const double target[3], const double up[3], double fov_y,
                     int W, int H, double* o, double* d) {
  double f[3], r[3], u[3];
  double n = 0;
  for (int a = 0; a < 3; ++a) { f[a] = target[a] - eye[a]; n += f[a] * f[a]; }
  n = sqrt(n);
  for (int a = 0; a < 3; ++a) f[a] /= n;
  r[0] = f[1] * up[2] - f[2] * up[1];
  r[1] = f[2] * up[0] - f[0] * up[2];
  r[2] = f[0] * up[1] - f[1] * up[0];
  n = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (int a = 0; a < 3; ++a) r[a] /= n;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  double th = tan(fov_y * M_PI / 360.0);
  double aspect = (double)W / (double)H;
  int64_t R = (int64_t)W * H;
  for (int row = 0; row < H; ++row)
    for (int col = 0; col < W; ++col) {
      int64_t i = (int64_t)row * W + col;
      double sx = 2.0 * (col + 0.5) / W - 1.0;
      double sy = 1.0 - 2.0 * (row + 0.5) / H;
      double v[3];
      double nn = 0;
      for (int a = 0; a < 3; ++a) {
        v[a] = f[a] + sx * th * aspect * r[a] + sy * th * u[a];
        nn += v[a] * v[a];
      }
      nn = sqrt(nn);
      for (int a = 0; a < 3; ++a) {
        o[a * R + i] = eye[a];
        d[a * R + i] = v[a] / nn;
      }
    }
}

/* ------------------------------------------------------------------ */
/* Sphere tracing with adaptive stepping (Sec. 3.4, Fig. 3; App. A.4)    */
/* ------------------------------------------------------------------ */
enum { ORC_MISS = 0, ORC_HIT = 1, ORC_MAX_STEPS = 2, ORC_FAR = 3, ORC_STALLED = 4, ORC_INVALID = 5 };

typedef struct {
  int max_steps;
  double delta;      /* hit threshold */
  double t_far;      /* far-plane clip */
  int osc_check;     /* stop when |d_k - d_{k-1}| < 6 delta */
  int analytic;      /* 1: exact SDF of the sphere below instead of the model */
  double sphere[4];  /* cx cy cz R */
  double margin_sdf; /* marginal if |dist - delta| <= margin_sdf * scale */
  double margin_t;   /* marginal if t within margin_t*(1+t) of a voxel bound */
} orc_trace_params;

/* SDF at x using the voxel `v` of depth Lt+1 and its ancestors (Sec. 3.4:
 * the parents of a traced voxel always exist).  Lt = lod, or lod+1 when
 * blending with alpha > 0. */
static double query_in_voxel(const orc_octree* t, const orc_model* M, int lod, double alpha, int pair_depth,
                             int64_t v, const double x[3], double* scale) {
  int Lp = alpha > 0.0 ? lod + 1 : lod;
  int m = M->m;
  int64_t vx, vy, vz;
  demorton3(t->code[pair_depth][v], &vx, &vy, &vz);
  double z[64], zn[64], psi[64];
  for (int k = 0; k < m; ++k) z[k] = zn[k] = 0.0;
  for (int l = 1; l <= Lp; ++l) {
    int s = (pair_depth - 1) - l; /* level l lives at depth l + 1 */
    int64_t cell[3] = {vx >> s, vy >> s, vz >> s};
    interp_level(t, M, l, cell, x, psi);
    if (l <= lod) for (int k = 0; k < m; ++k) z[k] += psi[k];
    else for (int k = 0; k < m; ++k) zn[k] = z[k] + psi[k];
  }
  double s0, s1;
  double d0 = decode(M, lod, x, z, &s0, NULL);
  if (alpha > 0.0) {
    double d1 = decode(M, lod + 1, x, zn, &s1, NULL);
    *scale = (1.0 - alpha) * s0 + alpha * s1;
    return (1.0 - alpha) * d0 + alpha * d1;
  }
  *scale = s0;
  return d0;
}

/*
 * Per ray, with its front-to-back pairs (pair_vox, t_in, t_out) at depth
 * Lt+1 (ray_off gives each ray's range):
 *   p = 0; t = t_in[0]; k = 0
 *   loop: skip pairs with t > t_out[p]; none left -> MISS;
 *         if t < t_in[p], advance t to t_in[p]; t > t_far -> FAR;
 *         k == max_steps -> MAX_STEPS; evaluate dist at o + t d; k++;
 *         dist < delta -> HIT; optional oscillation stop; t += dist.
 * Outputs t_hit (t at termination), status, steps and hit voxel, plus a
 * `marginal` flag for rays whose outcome could flip under small
 * perturbations (see orc_trace_params).
 */
static void trace_ray(const orc_octree* t, const orc_model* M, const float* o, const float* d, int64_t R,
                      int64_t i, int lod, double alpha, int pair_depth, const int32_t* pair_vox,
                      const float* t_in, const float* t_out, const int64_t* ray_off,
                      const orc_trace_params* prm, double* t_hit, uint8_t* status, int32_t* steps,
                      int32_t* hit_vox, uint8_t* marginal) {
  double oo[3] = {o[i], o[R + i], o[2 * R + i]};
  double dd[3] = {d[i], d[R + i], d[2 * R + i]};
  int64_t b = ray_off[i], e = ray_off[i + 1];
  int64_t p = b;
  double t_cur = b < e ? (double)t_in[b] : 0.0;
  int k = 0;
  double prev = INFINITY;
  uint8_t st = ORC_MISS, marg = 0;
  int32_t hv = -1;
  int bad = 0;
  for (int a = 0; a < 3; ++a) if (!isfinite(oo[a]) || !isfinite(dd[a])) bad = 1;
  if (bad) { st = ORC_INVALID; e = b; }
  for (;;) {
    if (bad) break;
    while (p < e && t_cur > (double)t_out[p]) {
      if (fabs(t_cur - (double)t_out[p]) <= prm->margin_t * (1.0 + fabs(t_cur))) marg = 1;
      ++p;
    }
    if (p < e && fabs(t_cur - (double)t_out[p]) <= prm->margin_t * (1.0 + fabs(t_cur))) marg = 1;
    if (p == e) { st = ORC_MISS; break; }
    if (t_cur < (double)t_in[p]) t_cur = (double)t_in[p];
    if (t_cur > prm->t_far) { st = ORC_FAR; break; }
    if (k == prm->max_steps) { st = ORC_MAX_STEPS; break; }
    double x[3] = {oo[0] + t_cur * dd[0], oo[1] + t_cur * dd[1], oo[2] + t_cur * dd[2]};
    double scale = 1.0, dist;
    if (prm->analytic) {
      double q0 = x[0] - prm->sphere[0], q1 = x[1] - prm->sphere[1], q2 = x[2] - prm->sphere[2];
      dist = sqrt(q0 * q0 + q1 * q1 + q2 * q2) - prm->sphere[3];
    } else {
      dist = query_in_voxel(t, M, lod, alpha, pair_depth, pair_vox[p], x, &scale);
    }
    ++k;
    if (fabs(dist - prm->delta) <= prm->margin_sdf * scale) marg = 1;
    if (dist < prm->delta) { st = ORC_HIT; hv = pair_vox[p]; break; }
    if (prm->osc_check && fabs(dist - prev) < 6.0 * prm->delta) { st = ORC_STALLED; break; }
    prev = dist;
    t_cur += dist;
  }
  t_hit[i] = t_cur;
  status[i] = st;
  steps[i] = k;
  hit_vox[i] = hv;
  if (marginal) marginal[i] = marg;
}

int orc_sphere_trace(const orc_octree* t, const orc_model* M, const float* o, const float* d, int64_t R,
                     int lod, double alpha, const int32_t* pair_vox, const float* t_in, const float* t_out,
                     const int64_t* ray_off, const orc_trace_params* prm, double* t_hit, uint8_t* status,
                     int32_t* steps, int32_t* hit_vox, uint8_t* marginal) {
  if (!prm->analytic && (lod < 1 || lod > M->num_lods || M->m > 64)) return -1;
  if (!prm->analytic && alpha > 0.0 && lod >= M->num_lods) return -1;
  int pair_depth = (alpha > 0.0 ? lod + 1 : lod) + 1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < R; ++i)
    trace_ray(t, M, o, d, R, i, lod, alpha, pair_depth, pair_vox, t_in, t_out, ray_off, prm, t_hit, status, steps,
              hit_vox, marginal);
  return 0;
}

/*
 * Per-pixel LOD selection by distance (Sec. 3.4, LOD Selection): the LOD
 * moves linearly from lod_near at distance d_near to lod_far at d_far and
 * is constant outside.  Evaluated in FP32 in this order (every operation
 * rounded, no fused multiply-add):
 *   u = (dist - d_near) / (d_far - d_near), clamped to [0, 1];
 *   L~ = lod_near + (lod_far - lod_near) * u, clamped to [min, max] of the
 *        two LODs (rounding may leave that range by an ulp);
 *   L* = floor(L~) and alpha = L~ - L*, except L* = num_lods, alpha = 0
 *   when L~ >= num_lods.
 */
void orc_lod_select(float d_near, float d_far, float lod_near, float lod_far, int num_lods, float dist,
                    float* lod_cont, int32_t* lod_int, float* alpha) {
  float u = (dist - d_near) / (d_far - d_near);
  if (u < 0.0f) u = 0.0f;
  if (u > 1.0f) u = 1.0f;
  float span = lod_far - lod_near;
  float prod = span * u;
  float L = lod_near + prod;
  float lo = lod_near < lod_far ? lod_near : lod_far, hi = lod_near < lod_far ? lod_far : lod_near;
  if (L < lo) L = lo; /* rounding may leave the range by an ulp */
  if (L > hi) L = hi;
  int Li = (int)floorf(L);
  float a = L - (float)Li;
  if (Li >= num_lods) { Li = num_lods; a = 0.0f; }
  *lod_cont = L;
  *lod_int = Li;
  *alpha = a;
}

/*
 * Sphere trace with a LOD and blend weight per ray (lod_pp, alpha_pp) over
 * hit lists at any depth pair_depth >= (lod + (alpha > 0)) + 1 for every
 * ray: the SDF of a ray is evaluated at its own LOD from the ancestors of
 * the pair's voxel.
 */
int orc_sphere_trace_pp(const orc_octree* t, const orc_model* M, const float* o, const float* d, int64_t R,
                        int pair_depth, const int32_t* lod_pp, const float* alpha_pp, const int32_t* pair_vox,
                        const float* t_in, const float* t_out, const int64_t* ray_off,
                        const orc_trace_params* prm, double* t_hit, uint8_t* status, int32_t* steps,
                        int32_t* hit_vox, uint8_t* marginal) {
  if (M->m > 64 || pair_depth < 2 || pair_depth > M->num_lods + 1) return -1;
  for (int64_t i = 0; i < R; ++i) {
    int need = lod_pp[i] + (alpha_pp[i] > 0.0f ? 1 : 0);
    if (lod_pp[i] < 1 || lod_pp[i] > M->num_lods || need > M->num_lods || need + 1 > pair_depth) return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < R; ++i)
    trace_ray(t, M, o, d, R, i, lod_pp[i], (double)alpha_pp[i], pair_depth, pair_vox, t_in, t_out, ray_off, prm,
              t_hit, status, steps, hit_vox, marginal);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Training objective (Eq. 4) and its gradient                          */
/* ------------------------------------------------------------------ */
/*
 * J = (1/P) sum_p sum_{L=1..Lmax} w_L (f_{theta_L}([x_p, z(x_p; L)]) - d_p)^2
 * with w_L = 1 (Eq. 4), or per-LOD weights (0/1 for the progressive
 * schedule of the training appendix: LODs not yet trainable have weight 0).
 * Reverse mode, per point and LOD L with g = 2 w_L (dhat_L - d)/P:
 *   dW2_L += g h,  db2_L += g,  ga = w2 . 1[a > 0] g,
 *   dW1_L += ga (x) [x; z_L],  db1_L += ga,  dz_L = W1_z^T ga,
 *   dpsi_l = sum_{L >= l} dz_L,  dZ_l[corner(v_l, j)] += w_j dpsi_l.
 * Absent voxels contribute nothing to feature gradients.
 * Gradients are written (not accumulated) into the caller's buffers, laid
 * out like the parameters.  sdf_all (nullable) receives dhat_L [Lmax][P].
 */
int orc_train_fwd_bwd_w(const orc_octree* t, const orc_model* M, const float* xs, const float* target,
                        int64_t P, const double* lod_weight, double* loss, double* const* dfeat,
                        double* const* dW1, double* const* db1, double* const* dw2, double* db2,
                        double* sdf_all) {
  int Lm = M->num_lods, m = M->m, H = M->hidden, din = din_of(M);
  if (Lm != t->num_lods || m > 64) return -1;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  /* per-thread accumulators, summed in thread order at the end */
  size_t dec_sz = (size_t)Lm * ((size_t)H * din + H + H + 1);
  size_t feat_sz = 0;
  size_t feat_off[ORC_MAXL];
  for (int l = 0; l < Lm; ++l) { feat_off[l] = feat_sz; feat_sz += (size_t)t->ncorner[l] * m; }
  double* acc = (double*)calloc((size_t)nth * (dec_sz + feat_sz + 1), sizeof(double));
  size_t stride = dec_sz + feat_sz + 1;
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* A = acc + (size_t)tid * stride;
    double* gW1 = A;
    double* gb1 = gW1 + (size_t)Lm * H * din;
    double* gw2 = gb1 + (size_t)Lm * H;
    double* gb2 = gw2 + (size_t)Lm * H;
    double* gF = gb2 + Lm;
    double* gloss = gF + feat_sz;
    double psi[ORC_MAXL][64], zL[ORC_MAXL][64], w[ORC_MAXL][8], dz[ORC_MAXL][64];
    int64_t corner[ORC_MAXL][8];
    int have[ORC_MAXL];
    double* pre = (double*)malloc(sizeof(double) * (size_t)H);
    double* ga = (double*)malloc(sizeof(double) * (size_t)H);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
      double x[3] = {xs[p], xs[P + p], xs[2 * P + p]};
      int ok = in_box(x);
      for (int l = 1; l <= Lm; ++l) {
        int64_t r = (int64_t)1 << (l + 1);
        int64_t cell[3] = {0, 0, 0};
        int64_t v = -1;
        if (ok) {
          for (int q = 0; q < 3; ++q) cell[q] = cell_of(x[q], r);
          v = voxel_index(t, l + 1, cell[0], cell[1], cell[2]);
        }
        have[l - 1] = v >= 0;
        for (int k = 0; k < m; ++k) psi[l - 1][k] = 0.0;
        if (v >= 0) {
          interp_level(t, M, l, cell, x, psi[l - 1]);
          double u[3];
          for (int a = 0; a < 3; ++a) {
            double lo = -1.0 + 2.0 * (double)cell[a] / (double)r;
            u[a] = (x[a] - lo) * (double)r / 2.0;
            if (u[a] < 0.0) u[a] = 0.0;
            if (u[a] > 1.0) u[a] = 1.0;
          }
          for (int j = 0; j < 8; ++j) {
            int bb[3] = {j & 1, (j >> 1) & 1, (j >> 2) & 1};
            double ww = 1.0;
            for (int a = 0; a < 3; ++a) ww *= bb[a] ? u[a] : 1.0 - u[a];
            w[l - 1][j] = ww;
            corner[l - 1][j] = corner_index(t, l, cell[0] + bb[0], cell[1] + bb[1], cell[2] + bb[2]);
          }
        }
        for (int k = 0; k < m; ++k) zL[l - 1][k] = (l > 1 ? zL[l - 2][k] : 0.0) + psi[l - 1][k];
      }
      for (int L = 1; L <= Lm; ++L) {
        const double* W1 = M->W1[L - 1];
        const double* b1 = M->b1[L - 1];
        const double* w2 = M->w2[L - 1];
        double out = M->b2[L - 1];
        for (int k = 0; k < H; ++k) {
          double a = b1[k];
          int col = 0;
          if (M->with_xyz) for (int q = 0; q < 3; ++q) a += W1[(size_t)k * din + col++] * x[q];
          for (int q = 0; q < m; ++q) a += W1[(size_t)k * din + col++] * zL[L - 1][q];
          pre[k] = a;
          out += w2[k] * (a > 0.0 ? a : 0.0);
        }
        if (sdf_all) sdf_all[(size_t)(L - 1) * P + p] = out;
        double res = out - (double)target[p];
        double wL = lod_weight ? lod_weight[L - 1] : 1.0;
        *gloss += wL * res * res / (double)P;
        double g = 2.0 * wL * res / (double)P;
        gb2[L - 1] += g;
        for (int q = 0; q < m; ++q) dz[L - 1][q] = 0.0;
        for (int k = 0; k < H; ++k) {
          double h = pre[k] > 0.0 ? pre[k] : 0.0;
          gw2[(size_t)(L - 1) * H + k] += g * h;
          ga[k] = pre[k] > 0.0 ? w2[k] * g : 0.0;
          gb1[(size_t)(L - 1) * H + k] += ga[k];
          double* row = gW1 + ((size_t)(L - 1) * H + k) * din;
          int col = 0;
          if (M->with_xyz) for (int q = 0; q < 3; ++q) row[col++] += ga[k] * x[q];
          for (int q = 0; q < m; ++q) {
            row[col] += ga[k] * zL[L - 1][q];
            dz[L - 1][q] += W1[(size_t)k * din + col] * ga[k];
            ++col;
          }
        }
      }
      /* dpsi_l = sum_{L >= l} dz_L, scattered to the level-l corners */
      for (int l = 1; l <= Lm; ++l) {
        if (!have[l - 1]) continue;
        double dpsi[64];
        for (int q = 0; q < m; ++q) {
          dpsi[q] = 0.0;
          for (int L = l; L <= Lm; ++L) dpsi[q] += dz[L - 1][q];
        }
        for (int j = 0; j < 8; ++j) {
          double* dst = gF + feat_off[l - 1] + (size_t)corner[l - 1][j] * m;
          for (int q = 0; q < m; ++q) dst[q] += w[l - 1][j] * dpsi[q];
        }
      }
    }
    free(pre);
    free(ga);
  }
  /* reduce in thread order */
  double* S = (double*)calloc(stride, sizeof(double));
  for (int th = 0; th < nth; ++th)
    for (size_t k = 0; k < stride; ++k) S[k] += acc[(size_t)th * stride + k];
  double* gW1 = S;
  double* gb1 = gW1 + (size_t)Lm * H * din;
  double* gw2 = gb1 + (size_t)Lm * H;
  double* gb2 = gw2 + (size_t)Lm * H;
  double* gF = gb2 + Lm;
  for (int L = 0; L < Lm; ++L) {
    if (dW1 && dW1[L]) memcpy(dW1[L], gW1 + (size_t)L * H * din, sizeof(double) * (size_t)H * din);
    if (db1 && db1[L]) memcpy(db1[L], gb1 + (size_t)L * H, sizeof(double) * (size_t)H);
    if (dw2 && dw2[L]) memcpy(dw2[L], gw2 + (size_t)L * H, sizeof(double) * (size_t)H);
    if (dfeat && dfeat[L]) memcpy(dfeat[L], gF + feat_off[L], sizeof(double) * (size_t)t->ncorner[L] * m);
  }
  if (db2) memcpy(db2, gb2, sizeof(double) * (size_t)Lm);
  if (loss) *loss = gF[feat_sz];
  free(S);
  free(acc);
  return 0;
}

int orc_train_fwd_bwd(const orc_octree* t, const orc_model* M, const float* xs, const float* target,
                      int64_t P, double* loss, double* const* dfeat, double* const* dW1,
                      double* const* db1, double* const* dw2, double* db2, double* sdf_all) {
  return orc_train_fwd_bwd_w(t, M, xs, target, P, NULL, loss, dfeat, dW1, db1, dw2, db2, sdf_all);
}

/* Loss only (Eq. 4), for finite-difference checks. */
int orc_loss(const orc_octree* t, const orc_model* M, const float* xs, const float* target, int64_t P,
             double* loss) {
  return orc_train_fwd_bwd(t, M, xs, target, P, loss, NULL, NULL, NULL, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------ */
/* Analytic shapes and the SDF surface sampler (training appendix)      */
/* ------------------------------------------------------------------ */
/*
 * Union of spheres (cx, cy, cz, R) and tori (cx, cy, cz, R, r, axis): the
 * minimum of the primitives' exact signed distances.  A torus with axis a
 * has its ring in the plane of the other two coordinates.
 */
double orc_shape_sdf(int ns, const double* sph, int nt, const double* tor, const double x[3]) {
  double best = INFINITY;
  for (int i = 0; i < ns; ++i) {
    const double* c = sph + 4 * i;
    double q0 = x[0] - c[0], q1 = x[1] - c[1], q2 = x[2] - c[2];
    double dist = sqrt(q0 * q0 + q1 * q1 + q2 * q2) - c[3];
    if (dist < best) best = dist;
  }
  for (int i = 0; i < nt; ++i) {
    const double* c = tor + 6 * i;
    double q[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    int a = (int)c[5];
    int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
    double ring = sqrt(q[u] * q[u] + q[v] * q[v]) - c[3];
    double dist = sqrt(ring * ring + q[a] * q[a]) - c[4];
    if (dist < best) best = dist;
  }
  return best;
}

int orc_shape_sdf_many(int ns, const double* sph, int nt, const double* tor, const float* xs, int64_t P,
                       double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < P; ++p) {
    double x[3] = {xs[p], xs[P + p], xs[2 * P + p]};
    out[p] = orc_shape_sdf(ns, sph, nt, tor, x);
  }
  return 0;
}

/*
 * SDF surface sampler: ray i starts at a uniform point of the box,
 * o = -1 + 2 (u0, u1, u2), with a uniform direction on the sphere,
 * z = 1 - 2 u3, phi = 2 pi u4, d = (sqrt(1 - z^2) cos phi,
 * sqrt(1 - z^2) sin phi, z); it is sphere traced with steps |SDF| from
 * t = 0 and hits when |SDF| < delta (the point is returned), misses when it
 * leaves the box or after max_steps.  u: [5][n] uniforms in [0, 1).
 * marginal (nullable) flags rays whose outcome could flip under rounding:
 * a step ending within margin_box of the box's faces, or with |SDF| within
 * margin_sdf of delta.
 */
int orc_sample_surface(int ns, const double* sph, int nt, const double* tor, const float* u, int64_t n,
                       int max_steps, double delta, double margin_box, double margin_sdf, double* pts, uint8_t* hit,
                       uint8_t* marginal) {
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double o[3], d[3];
    for (int a = 0; a < 3; ++a) o[a] = -1.0 + 2.0 * (double)u[(size_t)a * (size_t)n + (size_t)i];
    double z = 1.0 - 2.0 * (double)u[3 * (size_t)n + (size_t)i];
    double phi = two_pi * (double)u[4 * (size_t)n + (size_t)i];
    double rxy = sqrt(fmax(0.0, 1.0 - z * z));
    d[0] = rxy * cos(phi);
    d[1] = rxy * sin(phi);
    d[2] = z;
    double t = 0.0;
    uint8_t h = 0, mg = 0;
    double x[3] = {o[0], o[1], o[2]};
    for (int k = 0; k < max_steps; ++k) {
      for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
      int out = 0;
      for (int a = 0; a < 3; ++a) {
        if (fabs(x[a]) > 1.0) out = 1;
        if (fabs(fabs(x[a]) - 1.0) <= margin_box) mg = 1;
      }
      if (out) break;
      double sd = orc_shape_sdf(ns, sph, nt, tor, x);
      if (fabs(fabs(sd) - delta) <= margin_sdf) mg = 1;
      if (fabs(sd) < delta) { h = 1; break; }
      t += fabs(sd);
    }
    for (int a = 0; a < 3; ++a) pts[(size_t)a * (size_t)n + (size_t)i] = h ? x[a] : 0.0;
    hit[i] = h;
    if (marginal) marginal[i] = mg;
  }
  return 0;
}

/*
 * Training points in the 2:2:1 surface : near : uniform split of the
 * training appendix, interleaved so every run of five points holds the
 * ratio: point i with q = i / 5, c = i % 5 is
 *   c = 0, 1: surface sample S[2q + c];
 *   c = 2, 3: near sample S[2q + c - 2] + sigma * g, g a standard normal
 *             triple from Box-Muller on (u0, u1), (u2, u3);
 *   c = 4:    uniform -1 + 2 (u0, u1, u2);
 * with u = uni[.][i] ([4][N] uniforms in [0, 1]; a radius input u0 or u2
 * of 0 is read as 1).  The
 * surface samples S ([3][ns_pts]) are used cyclically.  The target is the
 * shape's SDF at the (float32) point.
 */
int orc_training_points(int ns, const double* sph, int nt, const double* tor, const double* S, int64_t ns_pts,
                        const float* uni, int64_t N, double sigma, float* xs, double* target) {
  if (ns_pts <= 0) return -1;
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    int64_t q = i / 5;
    int c = (int)(i % 5);
    double u[4];
    for (int a = 0; a < 4; ++a) u[a] = (double)uni[(size_t)a * (size_t)N + (size_t)i];
    double x[3];
    if (c < 4) {
      int64_t k = (2 * q + (c < 2 ? c : c - 2)) % ns_pts;
      for (int a = 0; a < 3; ++a) x[a] = S[(size_t)a * (size_t)ns_pts + (size_t)k];
      if (c >= 2) {
        double r1 = sqrt(-2.0 * log(u[0] > 0.0 ? u[0] : 1.0)), r2 = sqrt(-2.0 * log(u[2] > 0.0 ? u[2] : 1.0));
        double g0 = r1 * cos(two_pi * u[1]), g1 = r1 * sin(two_pi * u[1]), g2 = r2 * cos(two_pi * u[3]);
        x[0] += sigma * g0;
        x[1] += sigma * g1;
        x[2] += sigma * g2;
      }
    } else {
      for (int a = 0; a < 3; ++a) x[a] = -1.0 + 2.0 * u[a];
    }
    double xf[3];
    for (int a = 0; a < 3; ++a) {
      float f = (float)x[a];
      xs[(size_t)a * (size_t)N + (size_t)i] = f;
      xf[a] = (double)f;
    }
    target[i] = orc_shape_sdf(ns, sph, nt, tor, xf);
  }
  return 0;
}

