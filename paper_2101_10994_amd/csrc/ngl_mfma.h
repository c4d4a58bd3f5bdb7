// Wavefront-level decoder on the gfx950 matrix cores.
//
// The 64 lanes of a wavefront each hold one point: its position x and its
// summed feature z (FP32, Eq. 2).  The decoder's first layer for all 64 points
// is a [h x K] x [K x 64] product evaluated as 16x16 tiles on the matrix
// cores; ReLU, the second layer (a dot product with w2) and the cross-lane
// reduction follow in FP32.  Two forms share the structure:
//   DecBF16: v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation);
//   DecF32:  v_mfma_f32_16x16x4f32 (FP32 operands and accumulation).
// BF16 operand layouts (verified on gfx950):
//   A[i][k]: lane l holds i = l%16, k = 8*(l/16) + 0..7
//   B[k][j]: lane l holds j = l%16, k = 8*(l/16) + 0..7
//   D[i][j]: lane l holds j = l%16, i = 4*(l/16) + r, r = 0..3
// BF16 form: the weights are used as stored (BF16).  Every FP32 activation
// a is carried as a_hi + a_lo, a_hi = bf16(a), a_lo = bf16(a - a_hi) (about
// 16 significant bits), so the only rounding beyond FP32 accumulation is
// that representation error (relative 2^-16):
//   K-steps s < KZ: features 32s..32s+31 (zero padded), once with z_hi and
//     once with z_lo against the same weight fragment;
//   the last K-step: columns [x_hi(3), x_lo(3), 1, 1, 0...] against weights
//     [W1_x(3), W1_x(3), b1_hi, b1_lo, 0...] (position and bias split alike).
// The points' inputs are staged in LDS as FP32 rows and split while the B
// fragments are formed.
#pragma once

#include "ngl_device.h"

namespace ngl {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ inline uint32_t f32_to_bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two FP32 values as packed BF16 bits, `lo` in the low half (one
// v_cvt_pk_bf16_f32, round to nearest even).
__device__ inline uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

// Eight FP32 values split into BF16 high parts and BF16 residuals:
// v[i] = hi[i] + lo[i] up to the rounding of the residual (relative 2^-16).
__device__ inline void split_bf16x8(const float4 a, const float4 b, uint4& hi, uint4& lo) {
  hi = make_uint4(pack_bf16(a.x, a.y), pack_bf16(a.z, a.w), pack_bf16(b.x, b.y), pack_bf16(b.z, b.w));
  lo = make_uint4(pack_bf16(a.x - __uint_as_float(hi.x << 16), a.y - __uint_as_float(hi.x & 0xffff0000u)),
                  pack_bf16(a.z - __uint_as_float(hi.y << 16), a.w - __uint_as_float(hi.y & 0xffff0000u)),
                  pack_bf16(b.x - __uint_as_float(hi.z << 16), b.y - __uint_as_float(hi.z & 0xffff0000u)),
                  pack_bf16(b.z - __uint_as_float(hi.w << 16), b.w - __uint_as_float(hi.w & 0xffff0000u)));
}

// The last K-step's B row of a point: [x_hi(3), x_lo(3), 1, 1] as BF16
// (x = x_hi + x_lo to about 16 bits), or [1, 1, 0...] without the position.
template <bool XYZ>
__device__ inline uint4 pos_bias_row(const float x[3]) {
  if constexpr (XYZ) {
    const uint32_t h01 = pack_bf16(x[0], x[1]);
    const uint32_t t1 = pack_bf16(x[2], x[0] - __uint_as_float(h01 << 16));
    const uint32_t t2 = pack_bf16(x[1] - __uint_as_float(h01 & 0xffff0000u), x[2] - __uint_as_float(t1 << 16));
    return make_uint4(h01, t1, t2, 0x3f80u | 0x3f80u << 16);
  } else {
    return make_uint4(0x3f80u | 0x3f80u << 16, 0u, 0u, 0u);
  }
}

template <int M, bool XYZ>
struct MfmaShape {
  static constexpr int OFF = XYZ ? 3 : 0;
  static constexpr int KZ = (M + 31) / 32;   // K-steps over the features
  static constexpr int KS = KZ + 1;          // weight fragments per hidden tile (+ position/bias step)
  static constexpr int ROW = M + 4;          // staged FP32 row: z (M), x (3), pad; 16-byte multiple
  static constexpr int STAGE_BYTES = 64 * ROW * 4;
  static constexpr int frag_bytes(int H) { return (H / 16) * KS * 64 * 16; }
};

// One lane's A fragment (16 bytes) of decoder L for hidden tile h and K-step
// s: row i = 16h + lane%16, columns 8*(lane/16) + 0..7 of that step.  W1 is
// read from the model unless `packed` (the fragments in this order, from
// ngl_pack_decoders) is given.
template <int M, bool XYZ>
__device__ inline uint4 frag_bf16(const ngl_model& md, int L, int h, int s, int lane) {
  using S = MfmaShape<M, XYZ>;
  const int din = M + S::OFF;
  const uint16_t* W1 = static_cast<const uint16_t*>(md.W1[L - 1]);
  const float* b1 = md.b1[L - 1];
  const int i = 16 * h + (lane & 15);
  const int g = lane >> 4;
  uint32_t bits[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kk = 8 * g + q;
    uint32_t b = 0;
    if (s < S::KZ) {
      const int f = 32 * s + kk;
      if (f < M) b = W1[i * din + S::OFF + f];
    } else if (XYZ) {
      if (kk < 3) b = W1[i * din + kk];
      else if (kk < 6) b = W1[i * din + kk - 3];
      else if (kk == 6) b = f32_to_bf16_bits(b1[i]);
      else if (kk == 7) b = f32_to_bf16_bits(b1[i] - __uint_as_float(f32_to_bf16_bits(b1[i]) << 16));
    } else {
      if (kk == 0) b = f32_to_bf16_bits(b1[i]);
      else if (kk == 1) b = f32_to_bf16_bits(b1[i] - __uint_as_float(f32_to_bf16_bits(b1[i]) << 16));
    }
    bits[q] = b;
  }
  return make_uint4(bits[0] | bits[1] << 16, bits[2] | bits[3] << 16, bits[4] | bits[5] << 16,
                    bits[6] | bits[7] << 16);
}

// Block-cooperative: A fragments of decoder L (BF16 weights) into LDS, and
// its w2 (FP32).  frag: [H/16][KS][64] 16-byte fragments, copied from the
// pre-packed decoder when the model has one.
template <int M, bool XYZ>
__device__ inline void load_frags(const ngl_model& md, int L, uint4* frag, float* w2s) {
  using S = MfmaShape<M, XYZ>;
  const int H = md.hidden;
  const int n = (H / 16) * S::KS * 64;
  const uint4* packed = static_cast<const uint4*>(md.W1_packed[L - 1]);
  if (packed) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) frag[e] = packed[e];
  } else {
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const int s = (e >> 6) % S::KS;
      const int h = (e >> 6) / S::KS;
      frag[e] = frag_bf16<M, XYZ>(md, L, h, s, e & 63);
    }
  }
  for (int k = threadIdx.x; k < H; k += blockDim.x) w2s[k] = md.w2[L - 1][k];
}

// max(a, 0) as one integer max on the bit pattern (negative floats, -0
// included, are negative integers).  A NaN input may pass through; the
// decoders' inputs are finite for every defined result.
__device__ inline float relu_bits(float a) { return __int_as_float(max(__float_as_int(a), 0)); }

// Orders this wavefront's LDS writes before its later LDS reads.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage this lane's decoder input row (FP32: z, then x) into the
// wavefront's buffer.
template <int M, bool XYZ>
__device__ inline void stage_row(float* stage, const float x[3], const float* z) {
  using S = MfmaShape<M, XYZ>;
  float4* row = reinterpret_cast<float4*>(stage + (threadIdx.x & 63) * S::ROW);
#pragma unroll
  for (int q = 0; q < M / 4; ++q) row[q] = make_float4(z[4 * q], z[4 * q + 1], z[4 * q + 2], z[4 * q + 3]);
  row[M / 4] = XYZ ? make_float4(x[0], x[1], x[2], 0.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// stage_row in two parts, for rows whose features were gathered by other
// lanes: the slice [off, off + 8) of row `row`'s features, and the rest of
// this lane's own row (its position).
template <int M, bool XYZ>
__device__ inline void stage_slice8(float* stage, int row, int off, const float* v) {
  using S = MfmaShape<M, XYZ>;
  float4* w = reinterpret_cast<float4*>(stage + row * S::ROW + off);
  w[0] = make_float4(v[0], v[1], v[2], v[3]);
  w[1] = make_float4(v[4], v[5], v[6], v[7]);
}

template <int M, bool XYZ>
__device__ inline void stage_rest_row(float* stage, int r, const float x[3]) {
  using S = MfmaShape<M, XYZ>;
  float4* row = reinterpret_cast<float4*>(stage + r * S::ROW);
  row[M / 4] = XYZ ? make_float4(x[0], x[1], x[2], 0.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

template <int M, bool XYZ>
__device__ inline void stage_rest(float* stage, const float x[3]) {
  stage_rest_row<M, XYZ>(stage, threadIdx.x & 63, x);
}

// B fragments of one staged point for the BF16 form: for each feature
// K-step the high and low parts of features 32s + 8g..+7 (zero past M), and
// in lanes g = 0 the position/bias step.
template <int M, bool XYZ>
__device__ inline void bf16_b_frags(const float* row, int g, bf16x8 (&bh)[MfmaShape<M, XYZ>::KZ],
                                    bf16x8 (&bl)[MfmaShape<M, XYZ>::KZ], bf16x8& bp) {
  using S = MfmaShape<M, XYZ>;
#pragma unroll
  for (int s = 0; s < S::KZ; ++s) {
    const int f0 = 32 * s + 8 * g;
    uint4 hi = make_uint4(0u, 0u, 0u, 0u), lo = hi;
    if (f0 < M) {
      const float4* r = reinterpret_cast<const float4*>(row + f0);
      split_bf16x8(r[0], r[1], hi, lo);
    }
    bh[s] = __builtin_bit_cast(bf16x8, hi);
    bl[s] = __builtin_bit_cast(bf16x8, lo);
  }
  uint4 t = make_uint4(0u, 0u, 0u, 0u);
  if (g == 0) {
    const float4 xv = *reinterpret_cast<const float4*>(row + M);
    const float x[3] = {xv.x, xv.y, xv.z};
    t = pos_bias_row<XYZ>(x);
  }
  bp = __builtin_bit_cast(bf16x8, t);
}

// First layer on the matrix cores, second layer and reduction in FP32 for
// one tile of 16 staged points (rows[16][ROW]): lane l returns the output of
// point l%16 less b2 (all 64 lanes must call it).
template <int M, bool XYZ>
__device__ inline float tile_decode(const uint4* frag, const float* w2s, const float* rows, int H) {
  using S = MfmaShape<M, XYZ>;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, j = lane & 15;
  bf16x8 bh[S::KZ], bl[S::KZ], bp;
  bf16_b_frags<M, XYZ>(rows + j * S::ROW, g, bh, bl, bp);
  float part = 0.0f;
  for (int h = 0; h < H / 16; ++h) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < S::KZ; ++s) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, frag[(h * S::KS + s) * 64 + lane]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[s], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[s], acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, frag[(h * S::KS + S::KZ) * 64 + lane]),
                                                  bp, acc, 0, 0, 0);
    const float4 w = *reinterpret_cast<const float4*>(w2s + 16 * h + 4 * g);
    part = fmaf(w.x, relu_bits(acc[0]), part);
    part = fmaf(w.y, relu_bits(acc[1]), part);
    part = fmaf(w.z, relu_bits(acc[2]), part);
    part = fmaf(w.w, relu_bits(acc[3]), part);
  }
  // sum over the four row groups of the tile (lanes j, j+16, j+32, j+48)
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part;
}

// The decoder output for this lane's staged point of the wavefront's 64
// rows (all 64 lanes must call it).  `live` (wave-uniform) marks the lanes
// whose output is used: a 16-lane point tile without any is skipped (its
// lanes get b2).
template <int M, bool XYZ>
__device__ inline float wave_decode(const uint4* frag, const float* w2s, float b2, const float* stage, int H,
                                    uint64_t live) {
  using S = MfmaShape<M, XYZ>;
  const int g = (threadIdx.x & 63) >> 4;
  float mine = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (((live >> (16 * t)) & 0xffffull) == 0) continue;
    const float part = tile_decode<M, XYZ>(frag, w2s, stage + 16 * t * S::ROW, H);
    if (g == t) mine = part;
  }
  return b2 + mine;
}

// ---------------------------------------------------------------------------
// FP32 form.  v_mfma_f32_16x16x4f32 layouts (verified on gfx950):
//   A[i][k]: lane l holds i = l%16, k = l/16;  B[k][j]: j = l%16, k = l/16;
//   D as above.  Inputs per point: [x(3), z(m), 1] (zero padded to a multiple
//   of 4), weights [W1 | b1]: position and bias stay exact FP32.
// ---------------------------------------------------------------------------
template <int M, bool XYZ>
struct MfmaShape32 {
  static constexpr int OFF = XYZ ? 3 : 0;
  static constexpr int KP = ((M + OFF + 1) + 3) / 4 * 4;
  static constexpr int KS = KP / 4;
  static constexpr int ROW = KP + 1;  // odd row stride spreads LDS banks
  static constexpr int STAGE_BYTES = 64 * ROW * 4;
  static constexpr int frag_bytes(int H) { return (H / 16) * KS * 64 * 4; }
};

// Element e of decoder L's FP32 fragments [H/16][KS][64]: hidden row
// 16h + lane%16, input column 4s + lane/16 of [W1 | b1] (zero past it).
template <int M, bool XYZ>
__device__ inline float frag_f32(const ngl_model& md, int L, int e) {
  using S = MfmaShape32<M, XYZ>;
  const int din = M + S::OFF;
  const float* W1 = static_cast<const float*>(md.W1[L - 1]);
  const int lane = e & 63;
  const int s = (e >> 6) % S::KS;
  const int h = (e >> 6) / S::KS;
  const int i = 16 * h + (lane & 15);
  const int k = 4 * s + (lane >> 4);
  return k < din ? W1[i * din + k] : (k == din ? md.b1[L - 1][i] : 0.0f);
}

template <int M, bool XYZ>
__device__ inline void load_frags32(const ngl_model& md, int L, float* frag, float* w2s) {
  using S = MfmaShape32<M, XYZ>;
  const int H = md.hidden;
  const int n = (H / 16) * S::KS * 64;
  const float* packed = static_cast<const float*>(md.W1_packed[L - 1]);
  if (packed) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) frag[e] = packed[e];
  } else {
    for (int e = threadIdx.x; e < n; e += blockDim.x) frag[e] = frag_f32<M, XYZ>(md, L, e);
  }
  for (int k = threadIdx.x; k < H; k += blockDim.x) w2s[k] = md.w2[L - 1][k];
}

template <int M, bool XYZ>
__device__ inline void stage_row32(float* stage, const float x[3], const float* z) {
  using S = MfmaShape32<M, XYZ>;
  float* row = stage + (threadIdx.x & 63) * S::ROW;
#pragma unroll
  for (int k = 0; k < S::KP; ++k) {
    float v = 0.0f;
    if (k < S::OFF) v = x[k < 3 ? k : 0];
    else if (k < S::OFF + M) v = z[k - S::OFF < M && k >= S::OFF ? k - S::OFF : 0];
    else if (k == S::OFF + M) v = 1.0f;
    row[k] = v;
  }
}

template <int M, bool XYZ>
__device__ inline void stage_slice8_32(float* stage, int row, int off, const float* v) {
  using S = MfmaShape32<M, XYZ>;
  float* w = stage + row * S::ROW + S::OFF + off;
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = v[i];
}

template <int M, bool XYZ>
__device__ inline void stage_rest32_row(float* stage, int r, const float x[3]) {
  using S = MfmaShape32<M, XYZ>;
  float* row = stage + r * S::ROW;
#pragma unroll
  for (int k = 0; k < S::KP; ++k) {
    if (k < S::OFF) row[k] = x[k < 3 ? k : 0];
    else if (k == S::OFF + M) row[k] = 1.0f;
    else if (k > S::OFF + M) row[k] = 0.0f;
  }
}

template <int M, bool XYZ>
__device__ inline void stage_rest32(float* stage, const float x[3]) {
  stage_rest32_row<M, XYZ>(stage, threadIdx.x & 63, x);
}

template <int M, bool XYZ>
__device__ inline float tile_decode32(const float* frag, const float* w2s, const float* rows, int H) {
  using S = MfmaShape32<M, XYZ>;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, j = lane & 15;
  float b[S::KS];
#pragma unroll
  for (int s = 0; s < S::KS; ++s) b[s] = rows[j * S::ROW + 4 * s + g];
  float part = 0.0f;
  for (int h = 0; h < H / 16; ++h) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < S::KS; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(frag[(h * S::KS + s) * 64 + lane], b[s], acc, 0, 0, 0);
    const float4 w = *reinterpret_cast<const float4*>(w2s + 16 * h + 4 * g);
    part = fmaf(w.x, relu_bits(acc[0]), part);
    part = fmaf(w.y, relu_bits(acc[1]), part);
    part = fmaf(w.z, relu_bits(acc[2]), part);
    part = fmaf(w.w, relu_bits(acc[3]), part);
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part;
}

template <int M, bool XYZ>
__device__ inline float wave_decode32(const float* frag, const float* w2s, float b2, const float* stage, int H,
                                      uint64_t live) {
  using S = MfmaShape32<M, XYZ>;
  const int g = (threadIdx.x & 63) >> 4;
  float mine = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (((live >> (16 * t)) & 0xffffull) == 0) continue;
    const float part = tile_decode32<M, XYZ>(frag, w2s, stage + 16 * t * S::ROW, H);
    if (g == t) mine = part;
  }
  return b2 + mine;
}

// Decoder policies used by the kernels.
template <int M, bool XYZ>
struct DecBF16 {
  using Frag = uint4;
  using Stage = float;
  static constexpr int STAGE_BYTES = MfmaShape<M, XYZ>::STAGE_BYTES;
  static constexpr int STAGE_ELEMS = 64 * MfmaShape<M, XYZ>::ROW;
  static constexpr int frag_elems(int H) { return (H / 16) * MfmaShape<M, XYZ>::KS * 64; }
  static constexpr int frag_bytes(int H) { return MfmaShape<M, XYZ>::frag_bytes(H); }
  __device__ static void load(const ngl_model& md, int L, Frag* f, float* w2s) { load_frags<M, XYZ>(md, L, f, w2s); }
  __device__ static void stage(Stage* st, const float x[3], const float* z) { stage_row<M, XYZ>(st, x, z); }
  __device__ static void stage_slice(Stage* st, int row, int off, const float* v) {
    stage_slice8<M, XYZ>(st, row, off, v);
  }
  __device__ static void stage_rest(Stage* st, const float x[3]) { ngl::stage_rest<M, XYZ>(st, x); }
  __device__ static float decode(const Frag* f, const float* w2s, float b2, const Stage* st, int H,
                                 uint64_t live = ~0ull) {
    return wave_decode<M, XYZ>(f, w2s, b2, st, H, live);
  }
  // one 16-point tile (rows[16][ROW]): staging row r, and the decode
  static constexpr int TILE_ELEMS = 16 * MfmaShape<M, XYZ>::ROW;
  static constexpr int TILE_BYTES = 4 * TILE_ELEMS;
  __device__ static void tile_rest(Stage* rows, int r, const float x[3]) { stage_rest_row<M, XYZ>(rows, r, x); }
  template <int D>
  __device__ static void tile_slice(Stage* rows, int r, int off, const float* v) {
    float* w = rows + r * MfmaShape<M, XYZ>::ROW + off;
    if constexpr (D % 4 == 0) {
#pragma unroll
      for (int q = 0; q < D / 4; ++q)
        reinterpret_cast<float4*>(w)[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) w[i] = v[i];
    }
  }
  __device__ static float tile(const Frag* f, const float* w2s, const Stage* rows, int H) {
    return tile_decode<M, XYZ>(f, w2s, rows, H);
  }
};

template <int M, bool XYZ>
struct DecF32 {
  using Frag = float;
  using Stage = float;
  static constexpr int STAGE_BYTES = MfmaShape32<M, XYZ>::STAGE_BYTES;
  static constexpr int STAGE_ELEMS = 64 * MfmaShape32<M, XYZ>::ROW;
  static constexpr int frag_elems(int H) { return (H / 16) * MfmaShape32<M, XYZ>::KS * 64; }
  static constexpr int frag_bytes(int H) { return MfmaShape32<M, XYZ>::frag_bytes(H); }
  __device__ static void load(const ngl_model& md, int L, Frag* f, float* w2s) { load_frags32<M, XYZ>(md, L, f, w2s); }
  __device__ static void stage(Stage* st, const float x[3], const float* z) { stage_row32<M, XYZ>(st, x, z); }
  __device__ static void stage_slice(Stage* st, int row, int off, const float* v) {
    stage_slice8_32<M, XYZ>(st, row, off, v);
  }
  __device__ static void stage_rest(Stage* st, const float x[3]) { stage_rest32<M, XYZ>(st, x); }
  __device__ static float decode(const Frag* f, const float* w2s, float b2, const Stage* st, int H,
                                 uint64_t live = ~0ull) {
    return wave_decode32<M, XYZ>(f, w2s, b2, st, H, live);
  }
  static constexpr int TILE_ELEMS = 16 * MfmaShape32<M, XYZ>::ROW;
  static constexpr int TILE_BYTES = 4 * TILE_ELEMS;
  __device__ static void tile_rest(Stage* rows, int r, const float x[3]) { stage_rest32_row<M, XYZ>(rows, r, x); }
  template <int D>
  __device__ static void tile_slice(Stage* rows, int r, int off, const float* v) {
    float* w = rows + r * MfmaShape32<M, XYZ>::ROW + MfmaShape32<M, XYZ>::OFF + off;
#pragma unroll
    for (int i = 0; i < D; ++i) w[i] = v[i];
  }
  __device__ static float tile(const Frag* f, const float* w2s, const Stage* rows, int H) {
    return tile_decode32<M, XYZ>(f, w2s, rows, H);
  }
};

// LDS carve-up shared by the kernels that decode with a policy:
// [frag0][frag1 (blend only)][w2s0][w2s1][stage per wavefront].
template <class DEC>
struct DecLds {
  typename DEC::Frag* frag0;
  typename DEC::Frag* frag1;
  float* w2s0;
  float* w2s1;
  typename DEC::Stage* stage;  // this wavefront's staging rows
  // stage_elems: staging elements per wavefront (64 rows, or one 16-row tile)
  __device__ DecLds(char* smem, int H, bool blend, int stage_elems = DEC::STAGE_ELEMS) {
    frag0 = reinterpret_cast<typename DEC::Frag*>(smem);
    frag1 = frag0 + DEC::frag_elems(H);
    w2s0 = reinterpret_cast<float*>(frag1 + (blend ? DEC::frag_elems(H) : 0));
    w2s1 = w2s0 + H;
    stage = reinterpret_cast<typename DEC::Stage*>(w2s1 + H) + (threadIdx.x >> 6) * stage_elems;
  }
  __host__ __device__ static size_t fixed_bytes(int H, bool blend) {
    return size_t(DEC::frag_bytes(H)) * (blend ? 2 : 1) + 2 * sizeof(float) * size_t(H);
  }
};

#ifndef NGL_COOP_BATCH
#define NGL_COOP_BATCH 1
#endif

// One level of the cooperative gather for the wavefront's 64 points:
// round s gives group r the point q = (64/G) s + r, whose voxel, cell and
// position come from lane q (the cell is (cx, cy, cz) >> sh, or with
// PACKED the packed cell word in cx).  The corner ids of all rounds are
// loaded first, then the row slices a few rounds at a time, so most loads
// of a level are in flight together.  Absent voxels (v < 0) load voxel 0's
// rows and keep their accumulator; rounds whose points are all outside
// `live` (wave-uniform lane mask) are skipped.
template <int M, typename FT, int G, bool PACKED>
__device__ __forceinline__ void coop_level(const ngl_model& md, int l, int sh, int v, const float x[3], int cx, int cy,
                                           int cz, int r, int g, float (*acc)[M / G], uint64_t live = ~0ull) {
  constexpr int D = M / G, NQ = 64 / G;
  constexpr uint64_t QM = NQ == 64 ? ~0ull : ((1ull << NQ) - 1ull);
  int vq[G];
  int4 c0[G], c1[G];
#pragma unroll
  for (int s = 0; s < G; ++s) {
    vq[s] = __shfl(v, NQ * s + r, 64);
    if (((live >> (NQ * s)) & QM) == 0) continue;
    const int4* cp = reinterpret_cast<const int4*>(md.corners[l - 1] + size_t(vq[s] >= 0 ? vq[s] : 0) * 8);
    c0[s] = cp[0];
    c1[s] = cp[1];
  }
  constexpr int B = NGL_COOP_BATCH < G ? NGL_COOP_BATCH : G;  // rounds whose row slices are in flight together
#pragma unroll
  for (int h = 0; h < G / B; ++h) {
    float fv[B][8][D];
#pragma unroll
    for (int s2 = 0; s2 < B; ++s2) {
      const int s = h * B + s2;
      if (((live >> (NQ * s)) & QM) == 0) continue;
      const int cs[8] = {c0[s].x, c0[s].y, c0[s].z, c0[s].w, c1[s].x, c1[s].y, c1[s].z, c1[s].w};
#pragma unroll
      for (int j = 0; j < 8; ++j) load_slice<M, FT, D>(md.feat[l - 1], cs[j], g * D, fv[s2][j]);
    }
#pragma unroll
    for (int s2 = 0; s2 < B; ++s2) {
      const int s = h * B + s2;
      if (((live >> (NQ * s)) & QM) == 0) continue;
      const int q = NQ * s + r;
      float xq[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) xq[a] = __shfl(x[a], q, 64);
      int qx, qy, qz;
      if constexpr (PACKED) {
        const uint32_t c = uint32_t(__shfl(cx, q, 64));
        qx = cell_x(c), qy = cell_y(c), qz = cell_z(c);
      } else {
        qx = __shfl(cx, q, 64) >> sh, qy = __shfl(cy, q, 64) >> sh, qz = __shfl(cz, q, 64) >> sh;
      }
      float u[3];
      cell_local(l, qx, qy, qz, xq, u);
      float t[D];
#pragma unroll
      for (int i = 0; i < D; ++i) t[i] = acc[s][i];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float w = corner_weight(u, j);
#pragma unroll
        for (int i = 0; i < D; ++i) t[i] = fmaf(w, fv[s2][j][i], t[i]);
      }
#pragma unroll
      for (int i = 0; i < D; ++i) acc[s][i] = vq[s] >= 0 ? t[i] : acc[s][i];
    }
  }
}

// Shape of the cooperative gather: G = M/8 lanes per point, each holding 8
// feature elements (M is a multiple of 8).
template <int M>
struct CoopShape {
  static constexpr int D = 8;      // feature elements per lane (16 or 32 bytes of a row)
  static constexpr int G = M / D;  // lanes per point in a gather round
};

// Gathered slices into the staging rows: round s of group r is row
// (64/G) s + r.
template <class DEC, int G>
__device__ __forceinline__ void stage_slices(typename DEC::Stage* st, int r, int g, const float (*acc)[8]) {
#pragma unroll
  for (int s = 0; s < G; ++s) DEC::stage_slice(st, (64 / G) * s + r, 8 * g, acc[s]);
}

// Tile-wise cooperative gather: the wavefront gathers and decodes its 64
// points one 16-point tile at a time, the 4 lanes of group r = lane / 4
// serving point r of the tile, lane g = lane % 4 holding the M/4 feature
// elements [g M/4, g M/4 + M/4).  Only one tile's accumulators and one
// tile's staging rows are live, which keeps register and LDS use low enough
// for three to four wavefronts per SIMD.
template <int M>
struct TileShape {
  static constexpr int G = 4;      // lanes per point
  static constexpr int D = M / 4;  // feature elements per lane
};

// Level 1 (resolution 4, at most 5^3 corners) can be staged in LDS by the
// block: its corner rows are then read through the LDS, off the vector
// memory path that the other levels' rows load through.  Used with FP32
// features (measured slower with 16-bit features: l1_bytes is 0 for them).
constexpr int kL1MaxCorners = 125;
template <int M, typename FT>
constexpr size_t l1_bytes() {
  return std::is_same<FT, F32>::value ? size_t(kL1MaxCorners) * M * 4 : 0;
}
// Whole block; the caller synchronises before use.  Needs ncorner[0] <=
// kL1MaxCorners (l1_fits).
template <int M, typename FT>
__device__ inline void stage_l1(const ngl_model& md, void* dst) {
  const int n = int(md.ncorner[0] * int64_t(M) * (std::is_same<FT, F32>::value ? 4 : 2) / 16);
  const uint4* src = static_cast<const uint4*>(md.feat[0]);
  uint4* d = static_cast<uint4*>(dst);
  for (int e = threadIdx.x; e < n; e += blockDim.x) d[e] = src[e];
}
inline bool l1_fits(const ngl_model& md) { return md.ncorner[0] <= kL1MaxCorners && md.nvox[2] > 0; }

// load_slice from the LDS copy (read as LDS, not through a generic address).
template <int M, typename FT, int D>
__device__ __forceinline__ void load_slice_lds(const void* base, int c, int off, float* v) {
  typedef const __attribute__((address_space(3))) char* lptr;
  constexpr int ES = std::is_same<FT, F32>::value ? 4 : 2;
  constexpr int BYTES = D * ES;  // 4 to 32, a power of two
  constexpr int W = BYTES >= 16 ? 4 : BYTES / 4;  // 32-bit words per load
  constexpr int NL = BYTES >= 16 ? BYTES / 16 : 1;
  typedef uint32_t uvw __attribute__((ext_vector_type(W)));
  const lptr r = (lptr)(base) + uint32_t(c) * uint32_t(M * ES) + uint32_t(off * ES);
  uint32_t wv[NL * W];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const uvw f = *(const __attribute__((address_space(3))) uvw*)(r + 16 * q);
#pragma unroll
    for (int e = 0; e < W; ++e) wv[q * W + e] = f[e];
  }
  if constexpr (std::is_same<FT, F32>::value) {
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = __uint_as_float(wv[i]);
  } else {
#pragma unroll
    for (int e = 0; e < D / 2; ++e) {
      const uint32_t lo = wv[e] & 0xffffu, hi = wv[e] >> 16;
      v[2 * e] = std::is_same<FT, BF16>::value ? bf16_to_f32(lo) : f16_to_f32(lo);
      v[2 * e + 1] = std::is_same<FT, BF16>::value ? bf16_to_f32(hi) : f16_to_f32(hi);
    }
  }
}

// One level for this lane's group: voxel vq, cell (qx, qy, qz) at level l
// and position xq of the group's point; the slice of each corner row is
// accumulated in the order of interp_level.  A point without a voxel at the
// level (vq < 0) loads voxel 0's rows and keeps its accumulator.  With l1
// (wave-uniform), level 1's rows come from l1s, the LDS copy of stage_l1.
template <int M, typename FT>
__device__ __forceinline__ void tile_level(const ngl_model& md, int l, int vq, const float xq[3], int qx, int qy,
                                           int qz, int g, float* acc, const void* l1s = nullptr, bool l1 = false) {
  constexpr int D = TileShape<M>::D;
  const int4* cp = reinterpret_cast<const int4*>(md.corners[l - 1] + size_t(vq >= 0 ? vq : 0) * 8);
  const int4 c0 = cp[0], c1 = cp[1];
  const int cs[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
  float fv[8][D];
  if (l1_bytes<M, FT>() > 0 && l == 1 && l1) {
#pragma unroll
    for (int j = 0; j < 8; ++j) load_slice_lds<M, FT, D>(l1s, cs[j], g * D, fv[j]);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) load_slice<M, FT, D>(md.feat[l - 1], cs[j], g * D, fv[j]);
  }
  float u[3];
  cell_local(l, qx, qy, qz, xq, u);
  float t[D];
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = acc[i];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float w = corner_weight(u, j);
#pragma unroll
    for (int i = 0; i < D; ++i) t[i] = fmaf(w, fv[j][i], t[i]);
  }
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = vq >= 0 ? t[i] : acc[i];
}

}  // namespace ngl
