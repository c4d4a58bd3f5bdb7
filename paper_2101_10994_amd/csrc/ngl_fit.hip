// Fitting pieces of the training appendix on gfx950: the analytic union SDF
// of the synthetic shapes, the SDF surface sampler (sphere tracing of random
// rays), the 2:2:1 surface/near/uniform training set, and a fused Adam step
// over many tensors.  Random numbers are inputs (uniforms in [0, 1]).
#include "ngl_common.h"
#include "ngl_device.h"

#include <cmath>

namespace ngl {

constexpr int kFitBlock = 256;

// Union of spheres [cx, cy, cz, R] and tori [cx, cy, cz, R, r, axis]:
// minimum of the primitives' exact signed distances (FP32).
__device__ inline float shape_sdf(const ngl_shape& sh, float x0, float x1, float x2) {
  float best = __builtin_inff();
  for (int i = 0; i < sh.n_spheres; ++i) {
    const float* c = sh.spheres + 4 * i;
    const float q0 = x0 - c[0], q1 = x1 - c[1], q2 = x2 - c[2];
    best = fminf(best, sqrtf(q0 * q0 + q1 * q1 + q2 * q2) - c[3]);
  }
  for (int i = 0; i < sh.n_tori; ++i) {
    const float* c = sh.tori + 6 * i;
    const float q[3] = {x0 - c[0], x1 - c[1], x2 - c[2]};
    const int a = int(c[5]);
    const float qa = a == 0 ? q[0] : (a == 1 ? q[1] : q[2]);
    const float qu = a == 0 ? q[1] : q[0];
    const float qv = a == 2 ? q[1] : q[2];
    const float ring = sqrtf(qu * qu + qv * qv) - c[3];
    best = fminf(best, sqrtf(ring * ring + qa * qa) - c[4]);
  }
  return best;
}

__global__ __launch_bounds__(kFitBlock) void k_shape_sdf(ngl_shape sh, const float* __restrict__ x, int64_t P,
                                                         float* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * kFitBlock + threadIdx.x;
  if (p < P) out[p] = shape_sdf(sh, x[p], x[P + p], x[2 * P + p]);
}

// One candidate ray of the surface sampler: origin -1 + 2 (u0, u1, u2),
// direction (sqrt(1 - z^2) cos phi, sqrt(1 - z^2) sin phi, z) with
// z = 1 - 2 u3, phi = 2 pi u4; |SDF| steps from t = 0 until |SDF| < delta
// (hit), the box is left, or max_steps evaluations.
__device__ inline bool trace_sample(const ngl_shape& sh, const float* u, int64_t n, int64_t i, int max_steps,
                                    float delta, float x[3]) {
  float o[3], d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = -1.0f + 2.0f * u[a * n + i];
  const float z = 1.0f - 2.0f * u[3 * n + i];
  const float phi = 6.283185307179586f * u[4 * n + i];
  const float rxy = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  d[0] = rxy * cosf(phi);
  d[1] = rxy * sinf(phi);
  d[2] = z;
  float t = 0.0f;
  for (int k = 0; k < max_steps; ++k) {
    bool out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[a] = fmaf(t, d[a], o[a]);
      out = out || fabsf(x[a]) > 1.0f;
    }
    if (out) return false;
    const float s = shape_sdf(sh, x[0], x[1], x[2]);
    if (fabsf(s) < delta) return true;
    t += fabsf(s);
  }
  return false;
}

// Stable compaction of the hits, in ray order: per-block hit counts, one
// scan of the block counts, then each block writes its hits at its offset
// (ranks within a block from wavefront ballots and an LDS scan of the four
// wavefront counts).
struct SampleArgs {
  ngl_shape sh;
  const float* u;
  int64_t n;
  int max_steps;
  float delta;
  uint32_t* block_count;  // [blocks + 1]
  float* pts;             // [3][n]
  int64_t* count;         // device total
};

__global__ __launch_bounds__(kFitBlock) void k_sample_count(SampleArgs A) {
  __shared__ uint32_t wc[kFitBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kFitBlock + threadIdx.x;
  float x[3];
  const bool hit = i < A.n && trace_sample(A.sh, A.u, A.n, i, A.max_steps, A.delta, x);
  const uint64_t b = __ballot(hit);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = uint32_t(__popcll(b));
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kFitBlock / 64; ++w) s += wc[w];
    A.block_count[blockIdx.x] = s;
  }
}

// Exclusive scan of nb block counts in place (one block), total to *count.
__global__ __launch_bounds__(1024) void k_sample_scan(uint32_t* c, int64_t nb, int64_t* count) {
  __shared__ uint32_t part[1024];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = int64_t(threadIdx.x) * per;
  uint32_t s = 0;
  for (int64_t k = b0; k < b0 + per && k < nb; ++k) s += c[k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0u;
  for (int64_t k = b0; k < b0 + per && k < nb; ++k) {
    const uint32_t v = c[k];
    c[k] = run;
    run += v;
  }
  if (threadIdx.x == 1023) *count = int64_t(part[1023]);
}

__global__ __launch_bounds__(kFitBlock) void k_sample_emit(SampleArgs A) {
  __shared__ uint32_t wc[kFitBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kFitBlock + threadIdx.x;
  float x[3] = {0.0f, 0.0f, 0.0f};
  const bool hit = i < A.n && trace_sample(A.sh, A.u, A.n, i, A.max_steps, A.delta, x);
  const uint64_t b = __ballot(hit);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wc[w] = uint32_t(__popcll(b));
  __syncthreads();
  uint32_t off = A.block_count[blockIdx.x];
  for (int k = 0; k < w; ++k) off += wc[k];
  off += uint32_t(__popcll(b & ((1ull << lane) - 1ull)));
  if (hit) {
#pragma unroll
    for (int a = 0; a < 3; ++a) A.pts[a * A.n + off] = x[a];
  }
}

// Training set (2:2:1 surface, near, uniform, interleaved by i mod 5) in
// batch-major layout [N/B][3][B]; targets [N] (same order as the batches).
struct TrainSetArgs {
  ngl_shape sh;
  const float* S;   // [3][ns_stride] surface samples
  int64_t ns;       // samples used (cyclically)
  int64_t ns_stride;
  const float* uni; // [4][N]
  int64_t N;
  int64_t B;
  float sigma;
  float* xs;        // [N/B][3][B]
  float* target;    // [N]
};

__global__ __launch_bounds__(kFitBlock) void k_training_points(TrainSetArgs A) {
  const int64_t i = int64_t(blockIdx.x) * kFitBlock + threadIdx.x;
  if (i >= A.N) return;
  const int64_t q = i / 5;
  const int c = int(i % 5);
  float u[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) u[a] = A.uni[a * A.N + i];
  float x[3];
  if (c < 4) {
    const int64_t k = (2 * q + (c < 2 ? c : c - 2)) % A.ns;
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = A.S[a * A.ns_stride + k];
    if (c >= 2) {
      const float r1 = sqrtf(-2.0f * logf(u[0] > 0.0f ? u[0] : 1.0f));
      const float r2 = sqrtf(-2.0f * logf(u[2] > 0.0f ? u[2] : 1.0f));
      const float p1 = 6.283185307179586f * u[1], p2 = 6.283185307179586f * u[3];
      x[0] = fmaf(A.sigma, r1 * cosf(p1), x[0]);
      x[1] = fmaf(A.sigma, r1 * sinf(p1), x[1]);
      x[2] = fmaf(A.sigma, r2 * cosf(p2), x[2]);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmaf(2.0f, u[a], -1.0f);
  }
  const int64_t b = i / A.B, j = i % A.B;
#pragma unroll
  for (int a = 0; a < 3; ++a) A.xs[(b * 3 + a) * A.B + j] = x[a];
  A.target[i] = shape_sdf(A.sh, x[0], x[1], x[2]);
}

// Fused Adam over up to NGL_MAX_ADAM_TENSORS tensors; element e belongs to
// the tensor whose [start, start + numel) holds it.
struct AdamArgs {
  int n;
  float lr, beta1, beta2, eps, c1, c2;
  float* param[NGL_MAX_ADAM_TENSORS];
  const float* grad[NGL_MAX_ADAM_TENSORS];
  float* m[NGL_MAX_ADAM_TENSORS];
  float* v[NGL_MAX_ADAM_TENSORS];
  int64_t start[NGL_MAX_ADAM_TENSORS + 1];
};

__global__ __launch_bounds__(kFitBlock) void k_adam(AdamArgs A) {
  const int64_t total = A.start[A.n];
  for (int64_t e = int64_t(blockIdx.x) * kFitBlock + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * kFitBlock) {
    int lo = 0, hi = A.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.start[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int64_t k = e - A.start[lo];
    const float g = A.grad[lo][k];
    const float m = A.beta1 * A.m[lo][k] + (1.0f - A.beta1) * g;
    const float v = A.beta2 * A.v[lo][k] + (1.0f - A.beta2) * (g * g);
    A.m[lo][k] = m;
    A.v[lo][k] = v;
    A.param[lo][k] -= A.lr * (m * A.c1) / (sqrtf(v * A.c2) + A.eps);
  }
}

static int check_shape(const ngl_shape* sh) {
  NGL_REQUIRE(sh != nullptr, "shape is null");
  NGL_REQUIRE(sh->n_spheres >= 0 && sh->n_tori >= 0 && sh->n_spheres + sh->n_tori > 0,
              "shape needs at least one primitive");
  NGL_REQUIRE(sh->n_spheres == 0 || sh->spheres, "spheres is null");
  NGL_REQUIRE(sh->n_tori == 0 || sh->tori, "tori is null");
  return NGL_OK;
}

}  // namespace ngl

extern "C" {

int ngl_shape_sdf(const ngl_shape* shape, const float* x, int64_t P, float* sdf, void* stream) {
  int rc = ngl::check_shape(shape);
  if (rc) return rc;
  NGL_REQUIRE(P >= 0, "negative point count");
  if (P == 0) return NGL_OK;
  NGL_REQUIRE(x && sdf, "x or sdf is null");
  ngl::k_shape_sdf<<<unsigned((P + ngl::kFitBlock - 1) / ngl::kFitBlock), ngl::kFitBlock, 0,
                     (hipStream_t)stream>>>(*shape, x, P, sdf);
  NGL_LAUNCHED();
  return NGL_OK;
}

int ngl_sample_surface_workspace(int64_t n, size_t* bytes) {
  NGL_REQUIRE(bytes != nullptr && n >= 0, "bad arguments");
  *bytes = size_t(4) * size_t((n + ngl::kFitBlock - 1) / ngl::kFitBlock + 1);
  return NGL_OK;
}

int ngl_sample_surface(const ngl_shape* shape, const float* u, int64_t n, int32_t max_steps, float delta,
                       float* pts, int64_t* count, void* ws, size_t ws_bytes, void* stream) {
  int rc = ngl::check_shape(shape);
  if (rc) return rc;
  NGL_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "ray count out of range");
  NGL_REQUIRE(max_steps >= 0 && delta > 0.0f, "need max_steps >= 0 and delta > 0");
  NGL_REQUIRE(count != nullptr, "count is null");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nb = (n + ngl::kFitBlock - 1) / ngl::kFitBlock;
  NGL_REQUIRE(ws != nullptr && ws_bytes >= size_t(4) * size_t(nb + 1), "workspace too small");
  NGL_REQUIRE(n == 0 || (u && pts), "u or pts is null");
  ngl::SampleArgs A{*shape, u, n, int(max_steps), delta, static_cast<uint32_t*>(ws), pts, count};
  if (nb > 0) {
    ngl::k_sample_count<<<unsigned(nb), ngl::kFitBlock, 0, s>>>(A);
    NGL_LAUNCHED();
  }
  ngl::k_sample_scan<<<1, 1024, 0, s>>>(A.block_count, nb, count);
  NGL_LAUNCHED();
  if (nb > 0) {
    ngl::k_sample_emit<<<unsigned(nb), ngl::kFitBlock, 0, s>>>(A);
    NGL_LAUNCHED();
  }
  return NGL_OK;
}

int ngl_training_points(const ngl_shape* shape, const float* surface, int64_t n_surface, int64_t surface_stride,
                        const float* uniforms, int64_t N, int64_t batch, float sigma, float* x, float* target,
                        void* stream) {
  int rc = ngl::check_shape(shape);
  if (rc) return rc;
  NGL_REQUIRE(N >= 0 && batch > 0 && N % batch == 0, "N must be a multiple of batch > 0");
  NGL_REQUIRE(n_surface > 0 && surface_stride >= n_surface, "need surface samples (stride >= count > 0)");
  NGL_REQUIRE(std::isfinite(sigma) && sigma >= 0.0f, "sigma must be finite and >= 0");
  if (N == 0) return NGL_OK;
  NGL_REQUIRE(surface && uniforms && x && target, "null buffer");
  ngl::TrainSetArgs A{*shape, surface, n_surface, surface_stride, uniforms, N, batch, sigma, x, target};
  ngl::k_training_points<<<unsigned((N + ngl::kFitBlock - 1) / ngl::kFitBlock), ngl::kFitBlock, 0,
                           (hipStream_t)stream>>>(A);
  NGL_LAUNCHED();
  return NGL_OK;
}

int ngl_adam_step(const ngl_adam_params* p, int32_t n, float* const* param, const float* const* grad,
                  float* const* m, float* const* v, const int64_t* numel, void* stream) {
  NGL_REQUIRE(p != nullptr, "params is null");
  NGL_REQUIRE(n >= 0 && n <= NGL_MAX_ADAM_TENSORS, "tensor count %d outside 0..%d", n, NGL_MAX_ADAM_TENSORS);
  NGL_REQUIRE(p->step >= 1, "step counts from 1");
  NGL_REQUIRE(p->lr >= 0.0f && p->beta1 >= 0.0f && p->beta1 < 1.0f && p->beta2 >= 0.0f && p->beta2 < 1.0f &&
                  p->eps > 0.0f,
              "need lr >= 0, beta1 and beta2 in [0, 1), eps > 0");
  if (n == 0) return NGL_OK;
  NGL_REQUIRE(param && grad && m && v && numel, "null tensor list");
  ngl::AdamArgs A{};
  A.n = n;
  A.lr = p->lr;
  A.beta1 = p->beta1;
  A.beta2 = p->beta2;
  A.eps = p->eps;
  A.c1 = float(1.0 / (1.0 - std::pow(double(p->beta1), double(p->step))));
  A.c2 = float(1.0 / (1.0 - std::pow(double(p->beta2), double(p->step))));
  int64_t tot = 0;
  for (int i = 0; i < n; ++i) {
    NGL_REQUIRE(numel[i] >= 0, "numel[%d] < 0", i);
    NGL_REQUIRE(numel[i] == 0 || (param[i] && grad[i] && m[i] && v[i]), "tensor %d has a null buffer", i);
    A.param[i] = param[i];
    A.grad[i] = grad[i];
    A.m[i] = m[i];
    A.v[i] = v[i];
    A.start[i] = tot;
    tot += numel[i];
  }
  A.start[n] = tot;
  if (tot == 0) return NGL_OK;
  int64_t grid = (tot + ngl::kFitBlock - 1) / ngl::kFitBlock;
  if (grid > 4096) grid = 4096;
  ngl::k_adam<<<unsigned(grid), ngl::kFitBlock, 0, (hipStream_t)stream>>>(A);
  NGL_LAUNCHED();
  return NGL_OK;
}

}  // extern "C"
