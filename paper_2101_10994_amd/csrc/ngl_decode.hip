// Decoder-only evaluation: the per-LOD MLP of Eq. 2 applied to inputs
// [x, z] that the caller already holds (z = summed features, one row per
// point).  This is the query with the gather split off; it runs the same
// decoder forms:
//   * BF16 weights, hidden width 32/64/128: the first layer for 16 points at
//     a time on the matrix cores with every weight fragment held in
//     registers and the inputs loaded straight into the B-operand layout
//     (no LDS round trip), ReLU and the second layer on the accumulators;
//   * otherwise the LDS-staged wavefront decoders of the query kernels
//     (BF16 or FP32 matrix-core form) or the per-lane FP32 form.
#include "ngl_common.h"
#include "ngl_mfma.h"

namespace ngl {

struct DecodeArgs {
  const float* x;  // [3][P], or null without the position input
  const void* z;   // [P][m] rows, FP32 or BF16
  int64_t P;
  int lod;
  float* sdf;      // [P]
};

// Row p of z as FP32.
template <int M, typename ZT>
__device__ inline void load_row(const void* z, int64_t p, float* out) {
  if constexpr (std::is_same<ZT, BF16>::value) {
    const uint4* r = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(z) + p * M);
#pragma unroll
    for (int q = 0; q < M / 8; ++q) {
      const uint4 v = r[q];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        out[8 * q + 2 * e] = bf16_to_f32(w[e] & 0xffffu);
        out[8 * q + 2 * e + 1] = bf16_to_f32(w[e] >> 16);
      }
    }
  } else {
    const float4* r = reinterpret_cast<const float4*>(static_cast<const float*>(z) + p * M);
#pragma unroll
    for (int q = 0; q < M / 4; ++q) {
      const float4 v = r[q];
      out[4 * q] = v.x;
      out[4 * q + 1] = v.y;
      out[4 * q + 2] = v.z;
      out[4 * q + 3] = v.w;
    }
  }
}

// Register-resident BF16 form.  A wavefront takes U consecutive 16-point
// tiles at a time; lane (g = lane/16, j = lane%16) loads features
// 32s + 8g..+7 of point j of a tile for every K-step s, which is exactly its
// B fragment, and the lanes of g = 0 carry the tile's [x_hi, x_lo, 1, 1]
// step.  FP32 rows take a second pass per feature step with their BF16
// residuals (BF16 rows are exact and skip it).  The raw inputs of the
// wavefront's next U tiles are loaded before the current ones are decoded.
// NH = hidden/16.
template <int M, bool XYZ, typename ZT, int U>
struct RawTiles {
  static constexpr int KZ = MfmaShape<M, XYZ>::KZ;
  static constexpr int W = std::is_same<ZT, BF16>::value ? 1 : 2;  // 16-byte vectors per K-step and lane
  uint4 z[U][KZ][W];
  float x[U][3];
};

template <int M, bool XYZ, typename ZT, int U>
__device__ inline void load_tiles(const DecodeArgs& A, int64_t p0, RawTiles<M, XYZ, ZT, U>& R) {
  using RT = RawTiles<M, XYZ, ZT, U>;
  const int g = (threadIdx.x & 63) >> 4;
  const int64_t P = A.P;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t p = p0 + 16 * u;
    const int64_t pc = p < P ? p : P - 1;
#pragma unroll
    for (int s = 0; s < RT::KZ; ++s) {
      const int f0 = 32 * s + 8 * g;
#pragma unroll
      for (int w = 0; w < RT::W; ++w) R.z[u][s][w] = make_uint4(0u, 0u, 0u, 0u);
      if (f0 < M) {
        if constexpr (RT::W == 1) {
          R.z[u][s][0] = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(A.z) + pc * M + f0);
        } else {
          const uint4* r = reinterpret_cast<const uint4*>(static_cast<const float*>(A.z) + pc * M + f0);
          R.z[u][s][0] = r[0];
          R.z[u][s][1] = r[1];
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) R.x[u][a] = XYZ ? A.x[a * P + pc] : 0.0f;
  }
}

template <int M, bool XYZ, int NH, typename ZT, int U>
__device__ inline void decode_tiles(const DecodeArgs& A, int64_t p0, const RawTiles<M, XYZ, ZT, U>& R,
                                    const bf16x8 (&fr)[NH][MfmaShape<M, XYZ>::KS], const floatx4 (&w2v)[NH],
                                    float b2) {
  using S = MfmaShape<M, XYZ>;
  constexpr bool SPLIT = !std::is_same<ZT, BF16>::value;
  constexpr int NL = SPLIT ? S::KZ : 1;
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int64_t P = A.P;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    bf16x8 b[S::KS];
    bf16x8 bl[NL];
#pragma unroll
    for (int s = 0; s < S::KZ; ++s) {
      if constexpr (SPLIT) {
        uint4 hi, lo;
        split_bf16x8(__builtin_bit_cast(float4, R.z[u][s][0]), __builtin_bit_cast(float4, R.z[u][s][1]), hi, lo);
        b[s] = __builtin_bit_cast(bf16x8, hi);
        bl[s] = __builtin_bit_cast(bf16x8, lo);
      } else {
        b[s] = __builtin_bit_cast(bf16x8, R.z[u][s][0]);
      }
    }
    const uint4 t = pos_bias_row<XYZ>(R.x[u]);
    const bool keep = g == 0;
    b[S::KZ] = __builtin_bit_cast(bf16x8, make_uint4(keep ? t.x : 0u, keep ? t.y : 0u, keep ? t.z : 0u,
                                                     keep ? t.w : 0u));
    floatx4 acc[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      acc[h] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < S::KZ; ++s) {
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr[h][s], b[s], acc[h], 0, 0, 0);
        if constexpr (SPLIT) acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr[h][s], bl[s], acc[h], 0, 0, 0);
      }
      acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr[h][S::KZ], b[S::KZ], acc[h], 0, 0, 0);
    }
    float part = 0.0f;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
      for (int r = 0; r < 4; ++r) part = fmaf(w2v[h][r], relu_bits(acc[h][r]), part);
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    const int64_t p = p0 + 16 * u;
    if (g == 0 && p < P) A.sdf[p] = b2 + part;
  }
}

template <int M, bool XYZ, int NH, typename ZT, int U>
__global__ __launch_bounds__(256) void k_decode_rf(ngl_model md, DecodeArgs A) {
  using S = MfmaShape<M, XYZ>;
  __shared__ uint4 fl[NH * S::KS * 64];
  __shared__ float w2l[16 * NH];
  // fragments built cooperatively with a fixed trip count, so every
  // thread's weight loads are in flight together
  constexpr int NF = NH * S::KS * 64;
#pragma unroll
  for (int e0 = 0; e0 < NF; e0 += 256) {
    const int e = e0 + int(threadIdx.x);
    if (e < NF)
      fl[e] = md.W1_packed[A.lod - 1] ? static_cast<const uint4*>(md.W1_packed[A.lod - 1])[e]
                                      : frag_bf16<M, XYZ>(md, A.lod, (e >> 6) / S::KS, (e >> 6) % S::KS, e & 63);
  }
  if (threadIdx.x < 16 * NH) w2l[threadIdx.x] = md.w2[A.lod - 1][threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  bf16x8 fr[NH][S::KS];
  floatx4 w2v[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
#pragma unroll
    for (int s = 0; s < S::KS; ++s) fr[h][s] = __builtin_bit_cast(bf16x8, fl[(h * S::KS + s) * 64 + lane]);
#pragma unroll
    for (int r = 0; r < 4; ++r) w2v[h][r] = w2l[16 * h + 4 * g + r];
  }
  const float b2 = md.b2[A.lod - 1];
  const int64_t chunks = (A.P + 16 * U - 1) / (16 * U);
  const int64_t nw = int64_t(gridDim.x) * (blockDim.x >> 6);
  int64_t c = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  RawTiles<M, XYZ, ZT, U> next;
  if (c < chunks) load_tiles<M, XYZ, ZT, U>(A, c * (16 * U) + j, next);
  for (; c < chunks; c += nw) {
    const RawTiles<M, XYZ, ZT, U> cur = next;
    if (c + nw < chunks) load_tiles<M, XYZ, ZT, U>(A, (c + nw) * (16 * U) + j, next);
    decode_tiles<M, XYZ, NH, ZT, U>(A, c * (16 * U) + j, cur, fr, w2v, b2);
  }
}

// LDS-staged policy decoders (as in the query kernels), or the per-lane FP32
// form when MFMA is false.
template <int M, bool XYZ, typename ZT, int NW, class DEC, bool MFMA>
__global__ __launch_bounds__(64 * NW) void k_decode_lds(ngl_model md, DecodeArgs A) {
  extern __shared__ __align__(16) char smem[];
  const int H = md.hidden;
  DecLds<DEC> S(smem, H, false);
  if constexpr (MFMA) {
    DEC::load(md, A.lod, S.frag0, S.w2s0);
    __syncthreads();
  }
  const float b2 = md.b2[A.lod - 1];
  const int64_t P = A.P;
  for (int64_t base = int64_t(blockIdx.x) * (64 * NW); base < P; base += int64_t(gridDim.x) * (64 * NW)) {
    const int64_t p = base + threadIdx.x;
    const bool in = p < P;
    float x[3] = {0.0f, 0.0f, 0.0f};
    float z[M];
#pragma unroll
    for (int k = 0; k < M; ++k) z[k] = 0.0f;
    if (in) {
      if constexpr (XYZ) {
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = A.x[a * P + p];
      }
      load_row<M, ZT>(A.z, p, z);
    }
    float out;
    if constexpr (MFMA) {
      DEC::stage(S.stage, x, z);
      wave_lds_sync();
      out = DEC::decode(S.frag0, S.w2s0, b2, S.stage, H, __ballot(in));
      wave_lds_sync();
    } else {
      out = decode_f32<M, XYZ>(md, A.lod, x, z);
    }
    if (in) A.sdf[p] = out;
  }
}

#ifndef NGL_DECODE_TILES
#define NGL_DECODE_TILES 4
#endif
constexpr int kDecodeU = NGL_DECODE_TILES;  // 16-point tiles per wavefront iteration

// One resident wave of blocks (each block builds the fragments once, so the
// grid is sized to the occupancy and loops over the tiles).
template <int M, bool XYZ, typename ZT, int NH>
static int launch_rf(const ngl_model& md, const DecodeArgs& A, hipStream_t s) {
  const int resident = resident_grid(reinterpret_cast<const void*>(&k_decode_rf<M, XYZ, NH, ZT, kDecodeU>), 256, 0, 0);
  const int64_t T = (A.P + 15) / 16;
  int64_t grid = (T + 3) / 4;
  if (grid > resident) grid = resident;
  k_decode_rf<M, XYZ, NH, ZT, kDecodeU><<<unsigned(grid), 256, 0, s>>>(md, A);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, bool XYZ, typename ZT, class DEC, bool MFMA>
static int launch_lds(const ngl_model& md, const DecodeArgs& A, hipStream_t s) {
  const size_t lds = MFMA ? DecLds<DEC>::fixed_bytes(md.hidden, false) + 2 * DEC::STAGE_BYTES : 0;
  int64_t grid = (A.P + 127) / 128;
  if (grid > 4096) grid = 4096;
  k_decode_lds<M, XYZ, ZT, 2, DEC, MFMA><<<unsigned(grid), 128, lds, s>>>(md, A);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, bool XYZ, typename ZT>
static int run_decode(const ngl_model& md, const DecodeArgs& A, hipStream_t s) {
  if (md.w_dtype == NGL_BF16) {
    switch (md.hidden) {
      case 32: return launch_rf<M, XYZ, ZT, 2>(md, A, s);
      case 64: return launch_rf<M, XYZ, ZT, 4>(md, A, s);
      case 128: return launch_rf<M, XYZ, ZT, 8>(md, A, s);
      default: return launch_lds<M, XYZ, ZT, DecBF16<M, XYZ>, true>(md, A, s);
    }
  }
  if (option(NGL_OPT_F32_DECODER) == 1) return launch_lds<M, XYZ, ZT, DecF32<M, XYZ>, true>(md, A, s);
  return launch_lds<M, XYZ, ZT, DecF32<M, XYZ>, false>(md, A, s);
}

template <int M>
static int decode_m(const ngl_model& md, const DecodeArgs& A, int zt, hipStream_t s) {
  if (md.with_xyz)
    return zt == NGL_BF16 ? run_decode<M, true, BF16>(md, A, s) : run_decode<M, true, F32>(md, A, s);
  return zt == NGL_BF16 ? run_decode<M, false, BF16>(md, A, s) : run_decode<M, false, F32>(md, A, s);
}

// Decoder lod's fragments in the order load_frags / load_frags32 stage
// them (ngl_pack_decoders).
template <int M, bool XYZ>
__global__ void k_pack_decoder(ngl_model md, int lod, void* out, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (md.w_dtype == NGL_BF16) {
    using S = MfmaShape<M, XYZ>;
    static_cast<uint4*>(out)[e] = frag_bf16<M, XYZ>(md, lod, (e >> 6) / S::KS, (e >> 6) % S::KS, e & 63);
  } else {
    static_cast<float*>(out)[e] = frag_f32<M, XYZ>(md, lod, e);
  }
}

// Fragment elements and their size for one LOD of this model.
static void packed_shape(const ngl_model& m, int64_t& elems, size_t& elem_bytes) {
  const int off = m.with_xyz ? 3 : 0;
  if (m.w_dtype == NGL_BF16) {
    elems = int64_t(m.hidden / 16) * ((m.feat_dim + 31) / 32 + 1) * 64;
    elem_bytes = 16;
  } else {
    elems = int64_t(m.hidden / 16) * ((m.feat_dim + off + 1 + 3) / 4) * 64;
    elem_bytes = 4;
  }
}

static size_t packed_lod_bytes(const ngl_model& m) {
  int64_t n = 0;
  size_t eb = 0;
  packed_shape(m, n, eb);
  return (size_t(n) * eb + 255) / 256 * 256;
}

template <int M, bool XYZ>
static int pack_m(const ngl_model& m, char* out, hipStream_t s) {
  int64_t n = 0;
  size_t eb = 0;
  packed_shape(m, n, eb);
  const size_t per = packed_lod_bytes(m);
  for (int l = 1; l <= m.num_lods; ++l) {
    k_pack_decoder<M, XYZ><<<unsigned((n + 255) / 256), 256, 0, s>>>(m, l, out + size_t(l - 1) * per, int(n));
    NGL_LAUNCHED();
  }
  return NGL_OK;
}

template <int M>
static int pack_width(const ngl_model& m, char* out, hipStream_t s) {
  return m.with_xyz ? pack_m<M, true>(m, out, s) : pack_m<M, false>(m, out, s);
}

size_t packed_decoder_bytes(const ngl_model& m) { return packed_lod_bytes(m) * size_t(m.num_lods); }

}  // namespace ngl

extern "C" {

int ngl_packed_decoder_bytes(const ngl_model* m, size_t* bytes) {
  int rc = ngl::check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(bytes != nullptr, "bytes is null");
  *bytes = ngl::packed_decoder_bytes(*m);
  return NGL_OK;
}

int ngl_pack_decoders(ngl_model* m, void* packed, size_t bytes, void* stream) {
  int rc = ngl::check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(packed != nullptr, "packed is null");
  NGL_REQUIRE(reinterpret_cast<uintptr_t>(packed) % 256 == 0, "packed must be 256-byte aligned");
  const size_t need = ngl::packed_decoder_bytes(*m);
  NGL_REQUIRE(bytes >= need, "packed holds %zu bytes, %zu needed", bytes, need);
  ngl_model src = *m;
  for (int l = 0; l < NGL_MAX_LODS; ++l) src.W1_packed[l] = nullptr;
  char* out = static_cast<char*>(packed);
  hipStream_t s = (hipStream_t)stream;
  switch (m->feat_dim) {
    case 8: rc = ngl::pack_width<8>(src, out, s); break;
    case 16: rc = ngl::pack_width<16>(src, out, s); break;
    case 32: rc = ngl::pack_width<32>(src, out, s); break;
    case 64: rc = ngl::pack_width<64>(src, out, s); break;
    default: NGL_FAIL(NGL_E_UNSUPPORTED, "feat_dim %d not compiled (8, 16, 32, 64)", m->feat_dim);
  }
  if (rc) return rc;
  const size_t per = ngl::packed_decoder_bytes(*m) / size_t(m->num_lods);
  for (int l = 0; l < NGL_MAX_LODS; ++l) m->W1_packed[l] = l < m->num_lods ? out + size_t(l) * per : nullptr;
  return NGL_OK;
}

int ngl_decode_sdf(const ngl_model* m, int32_t lod, const float* x, const void* z, int32_t z_dtype, int64_t P,
                   float* sdf, void* stream) {
  int rc = ngl::check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(P >= 0, "negative point count");
  NGL_REQUIRE(lod >= 1 && lod <= m->num_lods, "lod %d outside 1..%d", lod, m->num_lods);
  NGL_REQUIRE(z_dtype == NGL_F32 || z_dtype == NGL_BF16, "z_dtype must be NGL_F32 or NGL_BF16");
  if (P == 0) return NGL_OK;
  NGL_REQUIRE(z != nullptr && sdf != nullptr, "z or sdf is null");
  NGL_REQUIRE(!m->with_xyz || x != nullptr, "the model reads the position: x is required");
  NGL_REQUIRE(reinterpret_cast<uintptr_t>(z) % 16 == 0, "z must be 16-byte aligned");
  ngl::DecodeArgs A{x, z, P, int(lod), sdf};
  hipStream_t s = (hipStream_t)stream;
  switch (m->feat_dim) {
    case 8: return ngl::decode_m<8>(*m, A, z_dtype, s);
    case 16: return ngl::decode_m<16>(*m, A, z_dtype, s);
    case 32: return ngl::decode_m<32>(*m, A, z_dtype, s);
    case 64: return ngl::decode_m<64>(*m, A, z_dtype, s);
    default: NGL_FAIL(NGL_E_UNSUPPORTED, "feat_dim %d not compiled (8, 16, 32, 64)", m->feat_dim);
  }
}

}  // extern "C"
