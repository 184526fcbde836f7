// Texturing pass (forward) and its backward.
//
// Paper: Rendering, Texturing Pass and eq. texture: for every selected slot
// x = o + D d, Tex = G(Delta * H(x)); eq. final: C = N + sum_j W_j Tex_j.
// Hash grid (Preliminaries, Instant-NGP; supplementary Implementation
// Details): per level l the point s_l x is interpolated trilinearly from the
// 8 hashed cell corners (MapPositive on the integer corner coordinates, then
// XOR with the primes 1, 2654435761, 805459861, masked to the table size),
// scaled by Delta_l = 1 - exp(-(f / (s_l D))^2 / (2 pi)) (eq. downweighting).
// The sample position gets a gradient through the interpolation
// (supplementary, Other details). MLP: hidden layers without bias, ReLU; the
// RGB head uses a sigmoid, the SH head's 48 outputs (degree 3) are decoded
// along the pixel's unit ray (Representation, Appearance).
//
// Work split: one wavefront handles 16 samples at a time. Lane (g, c), with
// g = lane / 16 and c = lane % 16, owns sample c and the four levels
// {2g, 2g+1, 8+2g, 9+2g}; its eight features are exactly the K-slice a 16x16
// matrix-core tile wants in that lane, so the MLP runs on the features in
// registers with no LDS round trip. The MLP is evaluated transposed
// (hidden x samples): each layer's output tile is already laid out as the
// next layer's B operand once its K index is permuted, and the weight
// operands are staged in LDS in the matching permuted order.
//   BF16 form: v_mfma_f32_16x16x32_bf16 (FP32 accumulate), activations
//              rounded to BF16 between layers.
//   FP32 form: v_mfma_f32_16x16x4_f32 (full FP32).
// The backward recomputes the features and the MLP, back-propagates through
// the MLP with the transposed weights, and forms the weight gradients from
// per-unit activation tiles staged in LDS (samples become the K index of the
// product), kept in MFMA accumulators for the whole launch and added to
// global memory once. It writes each sample's per-level feature gradients;
// the hash-grid gradient is then formed level by level without floating-point
// global atomics (scatter_bin files corner records into per-workgroup slabs,
// one launch per level over all cameras of a call; scatter_reduce sums each
// bucket's records in LDS).
#include <hip/hip_fp16.h>
#include <type_traits>
#include <math.h>

#include "nx_internal.h"

namespace nx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

constexpr int kTexThreads = 256;
constexpr int kWaves = kTexThreads / 64;
constexpr int kInPad = 32;

typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

// float -> bfloat16 bits, round to nearest even (gfx950 converts in hardware,
// two values per v_cvt_pk_bf16_f32).
__device__ __forceinline__ short f2bf(float x) { return __builtin_bit_cast(short, (__bf16)x); }
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const f2v v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2v));
}
__device__ __forceinline__ float bf2f(uint32_t b16) { return __uint_as_float(b16 << 16); }

template <int TDT>
__device__ __forceinline__ float2 load_pair(const void* table, uint32_t idx) {
  if constexpr (TDT == NX_F32) {
    return reinterpret_cast<const float2*>(table)[idx];
  } else {
    const uint32_t b = reinterpret_cast<const uint32_t*>(table)[idx];
    if constexpr (TDT == NX_F16) {
      return make_float2(__half2float(__ushort_as_half((unsigned short)(b & 0xFFFFu))),
                         __half2float(__ushort_as_half((unsigned short)(b >> 16))));
    } else {
      return make_float2(bf2f(b & 0xFFFFu), bf2f(b >> 16));
    }
  }
}

// MapPositive (supplementary, Implementation Details): z > 0 -> 2z - 1,
// z <= 0 -> -2z, i.e. the zigzag code of -z. Written with shifts: the
// compiler turns the two-armed select into a branch on the execution mask.
__device__ __forceinline__ uint32_t map_positive(int z) {
  const uint32_t n = 0u - (uint32_t)z;
  return (n << 1) ^ (uint32_t)((int32_t)n >> 31);
}

// Feature index (0..31) held by lane group g in element e of a layer-1 operand.
__device__ __forceinline__ int feat_index(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4); }
// Hidden index held by lane group g in element e of K-chunk h (BF16 form).
__device__ __forceinline__ int hid_index(int h, int g, int e) { return 16 * (2 * h + (e >> 2)) + 4 * g + (e & 3); }
// Level handled by lane group g in slot i (0..3): levels {2g, 2g+1, 8+2g, 9+2g}.
__device__ __forceinline__ int lane_level(int g, int i) { return (i < 2 ? 2 * g : 8 + 2 * g) + (i & 1); }

__device__ __forceinline__ f4 mfma_bf16_k32(s8 a, s8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}
__device__ __forceinline__ f4 mfma_bf16_k16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_f32_k4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 1/x from the hardware reciprocal (within 1 ulp): the texture path's
// divisions (ray setup, Delta_l and its derivative, the sigmoid head) feed
// FP32 arithmetic whose own rounding is of the same order, and every kernel
// that recomputes a quantity uses this same form.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <bool BF>
__device__ __forceinline__ float load_w(const void* w, int idx) {
  if constexpr (BF) {
    return bf2f(reinterpret_cast<const unsigned short*>(w)[idx]);
  } else {
    return reinterpret_cast<const float*>(w)[idx];
  }
}

// ------------------------------------------------------------------ weights in LDS
// Operand slots. BF16 form: a slot is 64 lanes x 8 bf16 (one 16x16x32 A
// operand). FP32 form: a slot is 64 lanes x 1 float (one 16x16x4 A operand).
// SH: the head has 48 outputs (degree-3 spherical-harmonics coefficients,
// three 16-row tiles) instead of 3 (one tile, rows 0..2 used).
template <bool BF, int HID, bool SH = false>
struct WLayout {
  static constexpr int MT = HID / 16;
  static constexpr int HT = HID / 32;
  static constexpr int OT = SH ? 3 : 1;        // head row tiles
  static constexpr int NOUT = SH ? 48 : 3;     // head rows used
  static constexpr int HO = (OT + 1) / 2;      // 32-deep K chunks of the head's transpose (BF16)
  // forward
  static constexpr int nA1 = BF ? MT : MT * 8;
  static constexpr int nA2 = BF ? MT * HT : MT * MT * 4;
  static constexpr int nA3 = BF ? HT * OT : MT * 4 * OT;
  // backward (transposed)
  static constexpr int nA3T = BF ? MT * HO : MT * 4 * OT;
  static constexpr int nA2T = BF ? MT * HT : MT * MT * 4;
  static constexpr int nA1T = BF ? 2 * HT : 2 * MT * 4;
  static constexpr int oA1 = 0, oA2 = oA1 + nA1, oA3 = oA2 + nA2;
  static constexpr int nFwd = oA3 + nA3;
  static constexpr int oA3T = nFwd, oA2T = oA3T + nA3T, oA1T = oA2T + nA2T;
  static constexpr int nAll = oA1T + nA1T;
  static constexpr int slot_bytes = BF ? 64 * 16 : 64 * 4;
};

// Value of element e of lane (g, c) in operand slot `slot`.
template <bool BF, int HID, bool SH>
__device__ float weight_operand(int slot, int g, int c, int e, const void* w1, const void* w2, const void* w3,
                                int in_dim) {
  using LY = WLayout<BF, HID, SH>;
  constexpr int NOUT = LY::NOUT;
  constexpr int MT = LY::MT;
  if constexpr (BF) {
    if (slot < LY::oA2) {  // A1[mt]
      const int mt = slot - LY::oA1, f = feat_index(g, e);
      return f < in_dim ? load_w<BF>(w1, (16 * mt + c) * in_dim + f) : 0.f;
    } else if (slot < LY::oA3) {  // A2[mt][h]
      const int q = slot - LY::oA2, mt = q / LY::HT, h = q % LY::HT;
      return load_w<BF>(w2, (16 * mt + c) * HID + hid_index(h, g, e));
    } else if (slot < LY::oA3T) {  // A3[ot][h]
      const int q = slot - LY::oA3, ot = q / LY::HT, h = q % LY::HT, row = 16 * ot + c;
      return row < NOUT ? load_w<BF>(w3, row * HID + hid_index(h, g, e)) : 0.f;
    } else if (slot < LY::oA2T) {  // A3T[mt][ho]
      const int q = slot - LY::oA3T, mt = q / LY::HO, ho = q % LY::HO, o = hid_index(ho, g, e);
      return o < NOUT ? load_w<BF>(w3, o * HID + 16 * mt + c) : 0.f;
    } else if (slot < LY::oA1T) {  // A2T[mt][h]
      const int q = slot - LY::oA2T, mt = q / LY::HT, h = q % LY::HT;
      return load_w<BF>(w2, hid_index(h, g, e) * HID + 16 * mt + c);
    } else {  // A1T[mz][h]
      const int q = slot - LY::oA1T, mz = q / LY::HT, h = q % LY::HT;
      const int f = 16 * mz + c;
      return f < in_dim ? load_w<BF>(w1, hid_index(h, g, e) * in_dim + f) : 0.f;
    }
  } else {
    if (slot < LY::oA2) {  // A1[mt][ks]
      const int q = slot - LY::oA1, mt = q / 8, ks = q % 8, f = feat_index(g, ks);
      return f < in_dim ? load_w<BF>(w1, (16 * mt + c) * in_dim + f) : 0.f;
    } else if (slot < LY::oA3) {  // A2[mt][mi][r]
      const int q = slot - LY::oA2, mt = q / (MT * 4), mi = (q / 4) % MT, r = q % 4;
      return load_w<BF>(w2, (16 * mt + c) * HID + 16 * mi + 4 * g + r);
    } else if (slot < LY::oA3T) {  // A3[ot][mi][r]
      const int q = slot - LY::oA3, ot = q / (MT * 4), mi = (q / 4) % MT, r = q % 4, row = 16 * ot + c;
      return row < NOUT ? load_w<BF>(w3, row * HID + 16 * mi + 4 * g + r) : 0.f;
    } else if (slot < LY::oA2T) {  // A3T[mt][ot][r]
      const int q = slot - LY::oA3T, mt = q / (LY::OT * 4), ot = (q / 4) % LY::OT, r = q % 4;
      const int o = 16 * ot + 4 * g + r;
      return o < NOUT ? load_w<BF>(w3, o * HID + 16 * mt + c) : 0.f;
    } else if (slot < LY::oA1T) {  // A2T[mt][mi][r]
      const int q = slot - LY::oA2T, mt = q / (MT * 4), mi = (q / 4) % MT, r = q % 4;
      return load_w<BF>(w2, (16 * mi + 4 * g + r) * HID + 16 * mt + c);
    } else {  // A1T[mz][mi][r]
      const int q = slot - LY::oA1T, mz = q / (MT * 4), mi = (q / 4) % MT, r = q % 4;
      const int f = 16 * mz + c;
      return f < in_dim ? load_w<BF>(w1, (16 * mi + 4 * g + r) * in_dim + f) : 0.f;
    }
  }
}

// Writes operand slots [0, n_slots) to dst (LDS or global memory); this
// thread handles elements first, first + stride, ...
template <bool BF, int HID, bool SH>
__device__ void stage_weights(unsigned char* dst, int n_slots, const void* w1, const void* w2, const void* w3,
                              int in_dim, int first = threadIdx.x, int stride = kTexThreads) {
  constexpr int per = BF ? 8 : 1;
  const int total = n_slots * 64 * per;
  for (int i = first; i < total; i += stride) {
    const int slot = i / (64 * per);
    const int lane = (i / per) % 64;
    const int e = i % per;
    const float v = weight_operand<BF, HID, SH>(slot, lane >> 4, lane & 15, e, w1, w2, w3, in_dim);
    if constexpr (BF) {
      reinterpret_cast<short*>(dst)[i] = f2bf(v);
    } else {
      reinterpret_cast<float*>(dst)[i] = v;
    }
  }
}

// The backward's operand slots in global memory, for widths whose slots do
// not fit in LDS next to the weight-gradient accumulators.
template <bool BF, int HID, bool SH>
__global__ void stage_weight_operands_kernel(unsigned char* wop, const void* w1, const void* w2, const void* w3,
                                             int in_dim) {
  stage_weights<BF, HID, SH>(wop, WLayout<BF, HID, SH>::nAll, w1, w2, w3, in_dim, blockIdx.x * blockDim.x + threadIdx.x,
                         gridDim.x * blockDim.x);
}

static_assert(WLayout<false, 128, true>::nAll * WLayout<false, 128, true>::slot_bytes <= (int)kWeightOperandBytes,
              "operand slots exceed their workspace section");
static_assert(WLayout<true, 128, true>::nAll * WLayout<true, 128, true>::slot_bytes <= (int)kWeightOperandBytes,
              "operand slots exceed their workspace section");

template <bool BF>
struct Operand;
template <>
struct Operand<true> {
  static __device__ __forceinline__ s8 get(const unsigned char* lds, int slot, int lane) {
    return reinterpret_cast<const s8*>(lds)[slot * 64 + lane];
  }
};
template <>
struct Operand<false> {
  static __device__ __forceinline__ float get(const unsigned char* lds, int slot, int lane) {
    return reinterpret_cast<const float*>(lds)[slot * 64 + lane];
  }
};

typedef uint32_t u4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s8 pack8(const float v[8]) {
  const u4v w = {pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]), pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7])};
  return __builtin_bit_cast(s8, w);
}
__device__ __forceinline__ s8 pack_tiles(f4 a, f4 b) {
  const u4v w = {pack_bf16x2(a[0], a[1]), pack_bf16x2(a[2], a[3]), pack_bf16x2(b[0], b[1]), pack_bf16x2(b[2], b[3])};
  return __builtin_bit_cast(s8, w);
}
// max(x, 0) as one integer max on the bit pattern (a float with the sign bit
// set is a negative integer; -0 becomes +0): fmaxf takes two instructions
// here, the first of which only quiets a signalling NaN.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ f4 relu4(f4 x) {
#pragma unroll
  for (int e = 0; e < 4; ++e) x[e] = relu(x[e]);
  return x;
}

// MLP forward for 16 samples: z[8] are this lane's features; h1/h2 receive
// the post-ReLU hidden tiles (rows 16 mt + 4 g + r); o receives the head
// tiles (rows 16 ot + 4 g + r; RGB logits in rows 0..2 of lane group 0, or
// the 48 SH coefficients).
template <bool BF, int HID, bool SH>
__device__ __forceinline__ void mlp_forward(const unsigned char* lds, int lane, const float z[8], f4* h1, f4* h2,
                                            f4* o) {
  using LY = WLayout<BF, HID, SH>;
  constexpr int MT = LY::MT;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  if constexpr (BF) {
    constexpr int HT = LY::HT;
    const s8 b0 = pack8(z);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) h1[mt] = relu4(mfma_bf16_k32(Operand<true>::get(lds, LY::oA1 + mt, lane), b0, zero));
    s8 b1[HT];
#pragma unroll
    for (int h = 0; h < HT; ++h) b1[h] = pack_tiles(h1[2 * h], h1[2 * h + 1]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f4 acc = zero;
#pragma unroll
      for (int h = 0; h < HT; ++h) acc = mfma_bf16_k32(Operand<true>::get(lds, LY::oA2 + mt * HT + h, lane), b1[h], acc);
      h2[mt] = relu4(acc);
    }
    s8 b2[HT];
#pragma unroll
    for (int h = 0; h < HT; ++h) b2[h] = pack_tiles(h2[2 * h], h2[2 * h + 1]);
#pragma unroll
    for (int ot = 0; ot < LY::OT; ++ot) {
      f4 acc = zero;
#pragma unroll
      for (int h = 0; h < HT; ++h) acc = mfma_bf16_k32(Operand<true>::get(lds, LY::oA3 + ot * HT + h, lane), b2[h], acc);
      o[ot] = acc;
    }
  } else {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f4 acc = zero;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) acc = mfma_f32_k4(Operand<false>::get(lds, LY::oA1 + mt * 8 + ks, lane), z[ks], acc);
      h1[mt] = relu4(acc);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f4 acc = zero;
#pragma unroll
      for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = mfma_f32_k4(Operand<false>::get(lds, LY::oA2 + (mt * MT + mi) * 4 + r, lane), h1[mi][r], acc);
      h2[mt] = relu4(acc);
    }
#pragma unroll
    for (int ot = 0; ot < LY::OT; ++ot) {
      f4 acc = zero;
#pragma unroll
      for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = mfma_f32_k4(Operand<false>::get(lds, LY::oA3 + (ot * MT + mi) * 4 + r, lane), h2[mi][r], acc);
      o[ot] = acc;
    }
  }
}

// ------------------------------------------------------------------ SH head
// Degree-3 real spherical harmonics of a unit direction (Representation,
// Appearance): the usual Cartesian forms with orthonormal constants.
__device__ __forceinline__ void sh_basis16(float x, float y, float z, float Y[16]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = 0.28209479177387814f;
  Y[1] = -0.4886025119029199f * y;
  Y[2] = 0.4886025119029199f * z;
  Y[3] = -0.4886025119029199f * x;
  Y[4] = 1.0925484305920792f * (x * y);
  Y[5] = -1.0925484305920792f * (y * z);
  Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
  Y[7] = -1.0925484305920792f * (x * z);
  Y[8] = 0.5462742152960396f * (xx - yy);
  Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
  Y[10] = 2.890611442640554f * (x * y) * z;
  Y[11] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
  Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
  Y[14] = 1.445305721320277f * z * (xx - yy);
  Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// Head row 16 ot + 4 g + r holds coefficient k = row / 3 of channel row % 3
// ([16][3] layout). For a fixed (ot, r) the lane group g picks one of four
// rows known at compile time: select Y_k and the channel without indexing a
// register array at run time.
template <int OT_, int R>
__device__ __forceinline__ float sh_row_basis(const float Y[16], int g) {
  constexpr int r0 = 16 * OT_ + R;
  return g == 0 ? Y[r0 / 3] : g == 1 ? Y[(r0 + 4) / 3] : g == 2 ? Y[(r0 + 8) / 3] : Y[(r0 + 12) / 3];
}
template <int OT_, int R>
__device__ __forceinline__ int sh_row_channel(int g) {
  constexpr int r0 = 16 * OT_ + R;
  return g == 0 ? r0 % 3 : g == 1 ? (r0 + 4) % 3 : g == 2 ? (r0 + 8) % 3 : (r0 + 12) % 3;
}

// The three channels before the clamp, sum_k Y_k a_{3k+c} + 0.5, for the 16
// samples of a wave (every lane of a sample's column gets them): each lane
// sums its 12 head rows, then the four lane groups add up.
__device__ __forceinline__ void sh_decode(const f4 o[3], const float Y[16], int g, float raw[3]) {
  float p[3] = {0.f, 0.f, 0.f};
#define NX_SH_ROW(OT_, R)                                                \
  {                                                                      \
    const float v = sh_row_basis<OT_, R>(Y, g) * o[OT_][R];              \
    const int ch = sh_row_channel<OT_, R>(g);                            \
    p[0] += ch == 0 ? v : 0.f;                                           \
    p[1] += ch == 1 ? v : 0.f;                                           \
    p[2] += ch == 2 ? v : 0.f;                                           \
  }
  NX_SH_ROW(0, 0) NX_SH_ROW(0, 1) NX_SH_ROW(0, 2) NX_SH_ROW(0, 3)
  NX_SH_ROW(1, 0) NX_SH_ROW(1, 1) NX_SH_ROW(1, 2) NX_SH_ROW(1, 3)
  NX_SH_ROW(2, 0) NX_SH_ROW(2, 1) NX_SH_ROW(2, 2) NX_SH_ROW(2, 3)
#undef NX_SH_ROW
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    p[ch] += __shfl_xor(p[ch], 16, 64);
    p[ch] += __shfl_xor(p[ch], 32, 64);
    raw[ch] = p[ch] + 0.5f;
  }
}

// dL/d(head rows) of this lane: Y_k dL/dc for the row's channel c.
__device__ __forceinline__ void sh_head_grad(const float Y[16], int g, const float dc[3], f4 dlog[3]) {
#define NX_SH_G(OT_, R)                                                  \
  {                                                                      \
    const int ch = sh_row_channel<OT_, R>(g);                            \
    const float d = ch == 0 ? dc[0] : (ch == 1 ? dc[1] : dc[2]);         \
    dlog[OT_][R] = sh_row_basis<OT_, R>(Y, g) * d;                       \
  }
  NX_SH_G(0, 0) NX_SH_G(0, 1) NX_SH_G(0, 2) NX_SH_G(0, 3)
  NX_SH_G(1, 0) NX_SH_G(1, 1) NX_SH_G(1, 2) NX_SH_G(1, 3)
  NX_SH_G(2, 0) NX_SH_G(2, 1) NX_SH_G(2, 2) NX_SH_G(2, 3)
#undef NX_SH_G
}

struct SampleInfo {
  int64_t s, p;
  bool valid, has;
  float D, W;
  float dx, dy, dz;  // world ray direction
};

// Sample (pixel c of the 4x4 patch at patch column qx, row qy; slot j).
// Lanes of a 16-lane row see the same slot of 16 neighbouring pixels, so at
// coarse levels they usually share a hash-grid cell. This part needs only the
// sample's depth: has = valid, W = 0.
__device__ __forceinline__ SampleInfo sample_ray_xy(const GridDev& gd, int K, int qx, int qy, int j, int c,
                                                    const float* depths) {
  SampleInfo si;
  const int px = 4 * qx + (c & 3);
  const int py = 4 * qy + (c >> 2);
  si.valid = px < gd.width && py < gd.height;
  si.p = si.valid ? (int64_t)py * gd.width + px : 0;
  si.s = si.p * K + j;
  si.has = si.valid;
  si.D = si.valid ? depths[si.s] : 1.0f;
  si.W = 0.0f;
  const float cx = ((float)px + 0.5f - gd.cx) * rcp(gd.fx);
  const float cy = ((float)py + 0.5f - gd.cy) * rcp(gd.fy);
  si.dx = gd.rot[0] * cx + gd.rot[1] * cy + gd.rot[2];
  si.dy = gd.rot[3] * cx + gd.rot[4] * cy + gd.rot[5];
  si.dz = gd.rot[6] * cx + gd.rot[7] * cy + gd.rot[8];
  return si;
}

// The same for patch q (patches tile the image row-major).
__device__ __forceinline__ SampleInfo sample_ray(const GridDev& gd, int K, int q, int j, int c,
                                                 const float* depths) {
  const int npx = (gd.width + 3) >> 2;
  const int qy = q / npx;
  return sample_ray_xy(gd, K, q - qy * npx, qy, j, c, depths);
}

__device__ __forceinline__ SampleInfo sample_info(const GridDev& gd, int K, int q, int j, int c,
                                                  const int32_t* ids, const float* depths, const float* weights) {
  SampleInfo si = sample_ray(gd, K, q, j, c, depths);
  const int id = si.valid ? ids[si.s] : -1;
  si.has = id >= 0;
  si.D = si.has ? si.D : 1.0f;
  si.W = si.has ? weights[si.s] : 0.0f;
  return si;
}

__host__ __device__ __forceinline__ int64_t n_patches(const GridDev& gd) {
  return (int64_t)((gd.width + 3) >> 2) * ((gd.height + 3) >> 2);
}

// Workgroup ids are dealt to the 8 XCDs in turn, and each XCD has its own L2.
// Renumbered this way, the workgroups on one XCD take consecutive work items
// (neighbouring patches, which share hash-grid cells) instead of every eighth.
__device__ __forceinline__ int64_t xcd_local_block() {
  const unsigned G = gridDim.x, b = blockIdx.x;
  return (G % 8u == 0u) ? (int64_t)(b % 8u) * (G / 8u) + b / 8u : (int64_t)b;
}

struct LevelGeom {
  int cx, cy, cz;  // lattice cell floor(s_l x)
  float frx, fry, frz;
  uint32_t hx[2], hy[2], hz[2];  // hashed corner coordinates per axis (before XOR)
  float delta, expo;             // Delta_l and exp(-kappa/D^2) = 1 - Delta_l
};

__device__ __forceinline__ LevelGeom level_geom(const GridLevel& L, const SampleInfo& si) {
  LevelGeom g;
  const float sD = L.scale * si.D;
  const float Px = fmaf(sD, si.dx, L.ofrac[0]);
  const float Py = fmaf(sD, si.dy, L.ofrac[1]);
  const float Pz = fmaf(sD, si.dz, L.ofrac[2]);
  const float fx = floorf(Px), fy = floorf(Py), fz = floorf(Pz);
  g.frx = Px - fx;
  g.fry = Py - fy;
  g.frz = Pz - fz;
  const int cx = L.oint[0] + (int)fx, cy = L.oint[1] + (int)fy, cz = L.oint[2] + (int)fz;
  g.cx = cx;
  g.cy = cy;
  g.cz = cz;
  g.hx[0] = map_positive(cx);
  g.hx[1] = map_positive(cx + 1);
  g.hy[0] = map_positive(cy) * kPrime1;
  g.hy[1] = map_positive(cy + 1) * kPrime1;
  g.hz[0] = map_positive(cz) * kPrime2;
  g.hz[1] = map_positive(cz + 1) * kPrime2;
  const float y = L.kappa * rcp(si.D * si.D);
  g.delta = -expm1f(-y);
  g.expo = 1.0f - g.delta;
  return g;
}

// One table entry (F = 2): a 16-bit pair is one 32-bit word, an FP32 pair two.
template <int TDT>
struct EntryT {
  using type = uint32_t;
};
template <>
struct EntryT<NX_F32> {
  using type = float2;
};

template <int TDT>
__device__ __forceinline__ typename EntryT<TDT>::type load_entry(const void* table, uint32_t idx) {
  if constexpr (TDT == NX_F32) {
    return reinterpret_cast<const float2*>(table)[idx];
  } else {
    return reinterpret_cast<const uint32_t*>(table)[idx];
  }
}

template <int TDT>
__device__ __forceinline__ float2 entry_value(typename EntryT<TDT>::type e) {
  if constexpr (TDT == NX_F32) {
    return e;
  } else if constexpr (TDT == NX_F16) {
    return make_float2(__half2float(__ushort_as_half((unsigned short)(e & 0xFFFFu))),
                       __half2float(__ushort_as_half((unsigned short)(e >> 16))));
  } else {
    return make_float2(bf2f(e & 0xFFFFu), bf2f(e >> 16));
  }
}

__device__ __forceinline__ uint32_t corner_hash(const LevelGeom& g, int b, uint32_t mask) {
  return (g.hx[b & 1] ^ g.hy[(b >> 1) & 1] ^ g.hz[(b >> 2) & 1]) & mask;
}

__device__ __forceinline__ float corner_weight(const LevelGeom& g, int b) {
  return ((b & 1) ? g.frx : 1.f - g.frx) * ((b & 2) ? g.fry : 1.f - g.fry) * ((b & 4) ? g.frz : 1.f - g.frz);
}

// A lane's four levels: whether each is active and its 8 corner entries.
// All 32 reads are issued before any is used (inactive levels read entry 0).
template <int TDT>
struct LaneEntries {
  typename EntryT<TDT>::type ent[4][8];
  bool act[4];
};

template <int TDT>
__device__ __forceinline__ void gather_lane(const GridDev& gd, const void* table, const SampleInfo& si, int g,
                                            uint32_t mask, LaneEntries<TDT>& E, float fraw[8], float delta[4],
                                            int32_t* cells_out, float* dcoef = nullptr) {
  LevelGeom lg[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int l = lane_level(g, i);
    E.act[i] = si.has && l < gd.levels;
    lg[i] = level_geom(gd.lv[l < gd.levels ? l : 0], si);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t base = (uint32_t)lane_level(g, i) << gd.log2_size;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint32_t idx = E.act[i] ? base + corner_hash(lg[i], b, mask) : 0u;
      E.ent[i][b] = load_entry<TDT>(table, idx);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float f0 = 0.f, f1 = 0.f;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const float w = corner_weight(lg[i], b);
      const float2 th = entry_value<TDT>(E.ent[i][b]);
      f0 = fmaf(w, th.x, f0);
      f1 = fmaf(w, th.y, f1);
    }
    fraw[2 * i] = E.act[i] ? f0 : 0.f;
    fraw[2 * i + 1] = E.act[i] ? f1 : 0.f;
    delta[i] = E.act[i] ? lg[i].delta : 0.f;
    if (dcoef) {
      // Depth derivative of this level's two features, as coefficients of the
      // feature gradients gz (applied once the MLP backward has produced them):
      // dL/dD = gz0 dcoef[2i] + gz1 dcoef[2i+1]. The sample point is
      // p = s (o + D d), so dp/dD = s d; the trilinear weight's derivative
      // along an axis is the product of the other two weights with sign + / -
      // for the upper / lower corner; Delta = 1 - exp(-kappa/D^2) gives
      // dDelta/dD = -(1 - Delta) 2 kappa / D^3. Each corner's weight is
      // differentiated along d first (one scalar per corner), so the entries
      // enter as in the interpolation: 16 multiply-adds on the stored values.
      const GridLevel& L = gd.lv[lane_level(g, i) < gd.levels ? lane_level(g, i) : 0];
      const float wx[2] = {1.f - lg[i].frx, lg[i].frx}, wy[2] = {1.f - lg[i].fry, lg[i].fry};
      const float wz[2] = {1.f - lg[i].frz, lg[i].frz};
      float ax0 = 0.f, ax1 = 0.f;  // sum over corners of entry x (d w_b / d p . d)
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const float gx = wy[by] * wz[bz], gy = wx[bx] * wz[bz], gz = wx[bx] * wy[by];
        const float dw = fmaf(bz ? gz : -gz, si.dz, fmaf(by ? gy : -gy, si.dy, (bx ? gx : -gx) * si.dx));
        const float2 th = entry_value<TDT>(E.ent[i][b]);
        ax0 = fmaf(dw, th.x, ax0);
        ax1 = fmaf(dw, th.y, ax1);
      }
      const float ds = lg[i].delta * L.scale;
      const float ddelta = -lg[i].expo * 2.0f * L.kappa * rcp(si.D * si.D * si.D);
      const float c0 = ds * ax0 + ddelta * f0;
      const float c1 = ds * ax1 + ddelta * f1;
      dcoef[2 * i] = E.act[i] ? c0 : 0.f;
      dcoef[2 * i + 1] = E.act[i] ? c1 : 0.f;
      // keep the coefficients here, so that the entries die now rather than
      // being carried to the end of the backward pass
      asm volatile("" : "+v"(dcoef[2 * i]), "+v"(dcoef[2 * i + 1]));
    }
    if (cells_out && E.act[i]) {
      int32_t* cp = cells_out + lane_level(g, i) * 3;
      cp[0] = lg[i].cx;
      cp[1] = lg[i].cy;
      cp[2] = lg[i].cz;
    }
  }
}

template <int TDT, bool BF, int HID, bool SH>
__global__ __launch_bounds__(kTexThreads, (HID <= 64 && BF && TDT != NX_F32 && !SH) ? 3 : 1) void texture_forward_kernel(GridDev gd, const void* __restrict__ table,
                                                                      const void* w1, const void* w2, const void* w3,
                                                                      int in_dim, int K, int log2K, int64_t n_samples,
                                                                      const int32_t* __restrict__ ids,
                                                                      const float* __restrict__ depths,
                                                                      const float* __restrict__ weights,
                                                                      const float* __restrict__ plain,
                                                                      float* __restrict__ tex,
                                                                      float* __restrict__ image,
                                                                      int32_t* __restrict__ cells,
                                                                      uint32_t* __restrict__ relu_masks,
                                                                      float* __restrict__ features) {
  using LY = WLayout<BF, HID, SH>;
  constexpr int MT = LY::MT;
  __shared__ __attribute__((aligned(16))) unsigned char lds[LY::nFwd * LY::slot_bytes];
  stage_weights<BF, HID, SH>(lds, LY::nFwd, w1, w2, w3, in_dim);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const uint32_t mask = (1u << gd.log2_size) - 1u;
  const int64_t n_q = n_patches(gd);
  for (int64_t q = xcd_local_block() * kWaves + wave; q < n_q; q += (int64_t)gridDim.x * kWaves) {
    float contrib[3] = {0.f, 0.f, 0.f};
    bool pix_valid = false;
    int64_t pix = 0;
    for (int j = 0; j < K; ++j) {
      const SampleInfo si = sample_info(gd, K, (int)q, j, c, ids, depths, weights);
      pix_valid = si.valid;
      pix = si.p;
      float z[8], fraw[8], delta[4];
      LaneEntries<TDT> E;
      gather_lane<TDT>(gd, table, si, g, mask, E, fraw, delta,
                       cells && si.valid ? cells + si.s * gd.levels * 3 : nullptr);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z[2 * i] = fraw[2 * i] * delta[i];
        z[2 * i + 1] = fraw[2 * i + 1] * delta[i];
        // the features are complete here: keep the table entries from
        // living on into the MLP
        asm volatile("" : "+v"(z[2 * i]), "+v"(z[2 * i + 1]));
      }
      if (features && si.valid) {
        float* fp = features + si.s * gd.levels * 2;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int l = lane_level(g, i);
          if (l < gd.levels) {
            fp[2 * l] = z[2 * i];
            fp[2 * l + 1] = z[2 * i + 1];
          }
        }
      }
      f4 h1[MT], h2[MT], o[LY::OT];
      mlp_forward<BF, HID, SH>(lds, lane, z, h1, h2, o);
      // the sample's texture: sigmoid of the RGB head (rows 0..2 of lane
      // group 0), or the SH coefficients decoded along the unit ray
      float tv[3];
      if constexpr (SH) {
        const float inv = rsqrtf(si.dx * si.dx + si.dy * si.dy + si.dz * si.dz);
        float Y[16], raw[3];
        sh_basis16(si.dx * inv, si.dy * inv, si.dz * inv, Y);
        sh_decode(o, Y, g, raw);
#pragma unroll
        for (int r = 0; r < 3; ++r) tv[r] = relu(raw[r]);
      } else {
#pragma unroll
        for (int r = 0; r < 3; ++r) tv[r] = rcp(1.0f + __expf(-o[0][r]));
      }
      if (relu_masks) {
        // Unit 16 mt + 4 g + r of this lane's sample -> word mt / 2, bit 16 (mt % 2) + 4 g + r.
        constexpr int NW = HID / 32;
        uint32_t w1[NW], w2[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          w1[w] = 0u;
          w2[w] = 0u;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t bit = 1u << (16 * (mt & 1) + 4 * g + r);
            if (h1[mt][r] > 0.f) w1[mt >> 1] |= bit;
            if (h2[mt][r] > 0.f) w2[mt >> 1] |= bit;
          }
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          w1[w] |= __shfl_xor(w1[w], 16, 64);
          w1[w] |= __shfl_xor(w1[w], 32, 64);
          w2[w] |= __shfl_xor(w2[w], 16, 64);
          w2[w] |= __shfl_xor(w2[w], 32, 64);
        }
        if (g == 0 && si.valid) {
          uint32_t* mp = relu_masks + si.s * (2 * NW);
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            mp[w] = si.has ? w1[w] : 0u;
            mp[NW + w] = si.has ? w2[w] : 0u;
          }
        }
      }
      if (g == 0 && si.valid) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const float t = si.has ? tv[r] : 0.0f;
          tex[si.s * 3 + r] = t;
          contrib[r] = fmaf(si.W, t, contrib[r]);
        }
      }
    }
    if (g == 0 && pix_valid) {
#pragma unroll
      for (int r = 0; r < 3; ++r) image[pix * 3 + r] = plain[pix * 3 + r] + contrib[r];
    }
  }
}

// Row r of a BF16 activation tile starts at element 16 tile_row(r): after
// every 4 rows of 16 samples (32 dwords) the tile skips 8 dwords, so that the
// four lane groups of a wave, which write rows 4 g + r of one column, reach
// four different bank groups instead of the same one. Only the BF16 tiles of
// hidden width 64 are padded: the FP32 tiles' 16-lane row writes use half the
// banks anyway, and at hidden width 128 the padding would cost a workgroup's
// place on the CU (the padded tiles need more than half its LDS).
template <bool BF, int HID>
constexpr bool kPadTiles = BF && HID <= 64;

template <bool PAD>
__device__ __forceinline__ int tile_row(int r) {
  return PAD ? r + (r >> 2) : r;
}

// Write a register tile set (rows 16 mt + 4 g + r, column c) into an LDS
// [rows][16] matrix.
template <bool BF, bool PAD>
__device__ __forceinline__ void put_rows(unsigned char* buf, int row, int c, float v) {
  if constexpr (BF) {
    reinterpret_cast<short*>(buf)[tile_row<PAD>(row) * 16 + c] = f2bf(v);
  } else {
    reinterpret_cast<float*>(buf)[row * 16 + c] = v;
  }
}

// Rows row0 .. row0 + 3 of column c from a register tile (rows 4 g + r):
// two values per conversion for BF16.
template <bool BF, bool PAD>
__device__ __forceinline__ void put_rows4(unsigned char* buf, int row0, int c, f4 v) {
  if constexpr (BF) {
    const uint32_t w01 = pack_bf16x2(v[0], v[1]), w23 = pack_bf16x2(v[2], v[3]);
    short* p = reinterpret_cast<short*>(buf) + tile_row<PAD>(row0) * 16 + c;  // row0 % 4 == 0
    p[0] = (short)(w01 & 0xFFFFu);
    p[16] = (short)(w01 >> 16);
    p[32] = (short)(w23 & 0xFFFFu);
    p[48] = (short)(w23 >> 16);
  } else {
    float* p = reinterpret_cast<float*>(buf) + row0 * 16 + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) p[16 * r] = v[r];
  }
}

// dW[out][in] += sum over 16 samples of Y[out][s] X[in][s] for output row
// tiles mo < NMO and column tiles mi < NMI: acc[mo * NMI + mi] += the
// 16-sample contribution (samples are the K index of the product), reading
// Y and X from LDS [rows][16] tiles.
template <bool BF, bool PAD, int NMO, int NMI>
__device__ __forceinline__ void weight_grad_accum(const unsigned char* Y, const unsigned char* X,
                                                  f4 (&acc)[NMO * NMI], int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int mo = 0; mo < NMO; ++mo) {
#pragma unroll
    for (int mi = 0; mi < NMI; ++mi) {
      f4& d = acc[mo * NMI + mi];
      if constexpr (BF) {
        // Y and X start at a row that is a multiple of 4, so relative rows pad alike
        const s4 a = *reinterpret_cast<const s4*>(reinterpret_cast<const short*>(Y) + tile_row<PAD>(16 * mo + c) * 16 +
                                                  4 * g);
        const s4 b = *reinterpret_cast<const s4*>(reinterpret_cast<const short*>(X) + tile_row<PAD>(16 * mi + c) * 16 +
                                                  4 * g);
        d = mfma_bf16_k16(a, b, d);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float a = reinterpret_cast<const float*>(Y)[(16 * mo + c) * 16 + 4 * q + g];
          const float b = reinterpret_cast<const float*>(X)[(16 * mi + c) * 16 + 4 * q + g];
          d = mfma_f32_k4(a, b, d);
        }
      }
    }
  }
}

// Per-unit activation tiles for the workgroup-cooperative weight gradients:
// [rows][16 samples] in the MLP's storage precision. Rows: Y3 = dL/dlogit
// (16, rows 0..2 used), X3 = h2, Y2 = dL/dh2, X2 = h1, Y1 = dL/dh1 (HID each),
// X1 = z (32).
template <bool BF, int HID, bool SH>
struct UnitTiles {
  static constexpr int elem = BF ? 2 : 4;
  static constexpr int oY3 = 0, oX3 = 16 * WLayout<BF, HID, SH>::OT, oY2 = oX3 + HID, oX2 = oY2 + HID,
                       oY1 = oX2 + HID, oX1 = oY1 + HID;
  static constexpr int rows = oX1 + kInPad;
  static constexpr int bytes = (kPadTiles<BF, HID> ? rows + rows / 4 : rows) * 16 * elem;
};

// WLDS: operand slots staged in LDS by every workgroup (hidden width 64), or
// read from wop in global memory (L2-resident; hidden width 128, whose slots
// do not fit in LDS next to the activation tiles).
//
// Weight gradients: every round each of the NW waves handles one unit (16
// samples at one slot of a 4x4-pixel patch) and writes its activation tiles
// to LDS; after a barrier every wave multiplies the tiles of all NW units into
// its own share of dW1, dW2 and dW3 (row tiles split across the waves), which
// it keeps in MFMA accumulator registers for the whole launch and adds to
// global memory once at the end. NW = 4, except BF16 at hidden width 128,
// which runs 8 waves (one workgroup per CU, 143 KB of tiles): a wave's share
// of the 128 x 128 dW2 then fits its registers beside the activations
// (with 4 waves it holds twice as much and spills).
constexpr int bwd_waves(bool bf, int hid) { return (bf && hid == 128) ? 8 : 4; }
// workgroups per CU the launch bounds ask for: two, or one where a workgroup
// is 8 waves or FP32 at hidden width 128
constexpr int bwd_blocks(bool bf, int hid) { return bwd_waves(bf, hid) == 8 ? 1 : ((hid <= 64 || bf) ? 2 : 1); }

template <int TDT, bool BF, int HID, bool SH, bool WLDS>
__global__ __launch_bounds__(64 * bwd_waves(BF, HID), bwd_blocks(BF, HID)) void texture_backward_kernel(
    GridDev gd, const void* __restrict__ table, const void* w1, const void* w2, const void* w3,
    const unsigned char* __restrict__ wop, int in_dim, int K,
    int log2K, int64_t n_samples, const int32_t* __restrict__ ids, const float* __restrict__ depths,
    const float* __restrict__ weights, const float* __restrict__ grad_image, const float* __restrict__ grad_tex,
    float2* __restrict__ feat_grad, float* g_w1, float* g_w2, float* g_w3, float* __restrict__ grad_depth) {
  using LY = WLayout<BF, HID, SH>;
  using UT = UnitTiles<BF, HID, SH>;
  constexpr int MT = LY::MT;
  constexpr int OT = LY::OT;
  constexpr int NW = bwd_waves(BF, HID);
  constexpr int RT = MT / NW;   // row tiles of dW1 / dW2 per wave
  constexpr int CT3 = MT / NW;  // column tiles of dW3 per wave
  static_assert(RT >= 1 && RT * NW == MT, "hidden width must be a multiple of 16 NW");
  static_assert(!WLDS || NW == kWaves, "weights are staged in LDS by 4-wave workgroups only");
  __shared__ __attribute__((aligned(16))) unsigned char lds[WLDS ? LY::nAll * LY::slot_bytes : 16];
  __shared__ __attribute__((aligned(16))) unsigned char tiles[NW * UT::bytes];
  const unsigned char* W;
  if constexpr (WLDS) {
    stage_weights<BF, HID, SH>(lds, LY::nAll, w1, w2, w3, in_dim);
    W = lds;
  } else {
    W = wop;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  unsigned char* T = tiles + wave * UT::bytes;  // this wave's unit
  constexpr bool PAD = kPadTiles<BF, HID>;
  auto row_ptr = [&](const unsigned char* base, int row) { return base + tile_row<PAD>(row) * 16 * UT::elem; };
  const uint32_t mask = (1u << gd.log2_size) - 1u;
  const int64_t n_q = n_patches(gd);
  const int64_t n_units = n_q * K;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 accW3[OT * CT3], accW2[RT * MT], accW1[RT * 2];
#pragma unroll
  for (int i = 0; i < OT * CT3; ++i) accW3[i] = zero;
#pragma unroll
  for (int i = 0; i < RT * MT; ++i) accW2[i] = zero;
#pragma unroll
  for (int i = 0; i < RT * 2; ++i) accW1[i] = zero;

  const int64_t first = xcd_local_block() * NW;
  const int64_t stride = (int64_t)gridDim.x * NW;
  const int64_t n_rounds = first < n_units ? (n_units - first + stride - 1) / stride : 0;
  for (int64_t round = 0; round < n_rounds; ++round) {
    if constexpr (!WLDS) {
      // operand slots come from global memory: keep their loads inside the
      // loop (hoisted, they would occupy hundreds of registers)
      asm volatile("" : "+s"(W));
    }
    const int64_t qj = first + round * stride + wave;
    if (qj < n_units) {
      const SampleInfo si = sample_info(gd, K, (int)(qj >> log2K), (int)(qj & (K - 1)), c, ids, depths, weights);
      // ---- recompute features (all corner reads in flight together)
      float z[8], fraw[8], delta[4], dcoef[8];
      LaneEntries<TDT> E;
      gather_lane<TDT>(gd, table, si, g, mask, E, fraw, delta, nullptr, dcoef);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z[2 * i] = fraw[2 * i] * delta[i];
        z[2 * i + 1] = fraw[2 * i + 1] * delta[i];
      }
      // ---- MLP forward, keeping activations
      f4 h1[MT], h2[MT], o[OT];
      mlp_forward<BF, HID, SH>(W, lane, z, h1, h2, o);
      // ---- head: dL/d(head rows): RGB logits in rows 0..2 of lane group 0,
      // or the 48 SH coefficients (every lane group holds 12 of them)
      f4 dlog[OT];
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) dlog[ot] = zero;
      if constexpr (SH) {
        const float inv = rsqrtf(si.dx * si.dx + si.dy * si.dy + si.dz * si.dz);
        float Y[16], raw[3];
        sh_basis16(si.dx * inv, si.dy * inv, si.dz * inv, Y);
        sh_decode(o, Y, g, raw);
        if (si.has) {
          float dc[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            float dt = si.W * grad_image[si.p * 3 + r];
            if (grad_tex) dt += grad_tex[si.s * 3 + r];
            dc[r] = raw[r] > 0.0f ? dt : 0.0f;
          }
          sh_head_grad(Y, g, dc, dlog);
        }
      } else {
        if (g == 0 && si.has) {
          const float g0 = grad_image[si.p * 3], g1 = grad_image[si.p * 3 + 1], g2 = grad_image[si.p * 3 + 2];
          const float gi[3] = {g0, g1, g2};
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const float t = rcp(1.0f + __expf(-o[0][r]));
            float dt = si.W * gi[r];
            if (grad_tex) dt += grad_tex[si.s * 3 + r];
            dlog[0][r] = dt * t * (1.0f - t);
          }
        }
      }
      // ---- MLP backward, layer by layer; each layer's two weight-gradient
      // factors go to this wave's tiles as soon as they exist, so the
      // activations die early (h2 after layer 3, dH2 and h1 after layer 2).
      f4 dzt[2];
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) put_rows4<BF, PAD>(T, UT::oY3 + 16 * ot + 4 * g, c, dlog[ot]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) put_rows4<BF, PAD>(T, UT::oX3 + 16 * mt + 4 * g, c, h2[mt]);
      f4 dh2[MT];
      if constexpr (BF) {
        constexpr int HO = LY::HO;
        s8 bd[HO];
#pragma unroll
        for (int ho = 0; ho < HO; ++ho) bd[ho] = pack_tiles(dlog[2 * ho], 2 * ho + 1 < OT ? dlog[2 * ho + 1] : zero);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          f4 a = zero;
#pragma unroll
          for (int ho = 0; ho < HO; ++ho) a = mfma_bf16_k32(Operand<true>::get(W, LY::oA3T + mt * HO + ho, lane), bd[ho], a);
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = h2[mt][r] > 0.f ? a[r] : 0.f;
          dh2[mt] = a;
        }
      } else {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          f4 a = zero;
#pragma unroll
          for (int ot = 0; ot < OT; ++ot)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              a = mfma_f32_k4(Operand<false>::get(W, LY::oA3T + (mt * OT + ot) * 4 + r, lane), dlog[ot][r], a);
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = h2[mt][r] > 0.f ? a[r] : 0.f;
          dh2[mt] = a;
        }
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        put_rows4<BF, PAD>(T, UT::oY2 + 16 * mt + 4 * g, c, dh2[mt]);
        put_rows4<BF, PAD>(T, UT::oX2 + 16 * mt + 4 * g, c, h1[mt]);
      }
      f4 dh1[MT];
      if constexpr (BF) {
        constexpr int HT = LY::HT;
        s8 b2[HT];
#pragma unroll
        for (int h = 0; h < HT; ++h) b2[h] = pack_tiles(dh2[2 * h], dh2[2 * h + 1]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          f4 a = zero;
#pragma unroll
          for (int h = 0; h < HT; ++h) a = mfma_bf16_k32(Operand<true>::get(W, LY::oA2T + mt * HT + h, lane), b2[h], a);
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = h1[mt][r] > 0.f ? a[r] : 0.f;
          dh1[mt] = a;
        }
      } else {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          f4 a = zero;
#pragma unroll
          for (int mi = 0; mi < MT; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              a = mfma_f32_k4(Operand<false>::get(W, LY::oA2T + (mt * MT + mi) * 4 + r, lane), dh2[mi][r], a);
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = h1[mt][r] > 0.f ? a[r] : 0.f;
          dh1[mt] = a;
        }
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) put_rows4<BF, PAD>(T, UT::oY1 + 16 * mt + 4 * g, c, dh1[mt]);
#pragma unroll
      for (int e = 0; e < 8; ++e) put_rows<BF, PAD>(T, UT::oX1 + feat_index(g, e), c, z[e]);
      if constexpr (BF) {
        constexpr int HT = LY::HT;
        s8 b1[HT];
#pragma unroll
        for (int h = 0; h < HT; ++h) b1[h] = pack_tiles(dh1[2 * h], dh1[2 * h + 1]);
#pragma unroll
        for (int mz = 0; mz < 2; ++mz) {
          f4 a = zero;
#pragma unroll
          for (int h = 0; h < HT; ++h) a = mfma_bf16_k32(Operand<true>::get(W, LY::oA1T + mz * HT + h, lane), b1[h], a);
          dzt[mz] = a;
        }
      } else {
#pragma unroll
        for (int mz = 0; mz < 2; ++mz) {
          f4 a = zero;
#pragma unroll
          for (int mi = 0; mi < MT; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              a = mfma_f32_k4(Operand<false>::get(W, LY::oA1T + (mz * MT + mi) * 4 + r, lane), dh1[mi][r], a);
          dzt[mz] = a;
        }
      }
      // ---- per-level feature gradients (distributed over the cell corners by
      // the hash-scatter kernel) and the depth gradient through the sample
      // position and Delta_l
      float dD = 0.f;
      const int64_t nqK = n_q * K;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int l = lane_level(g, i);
        const float gz0 = i < 2 ? dzt[0][2 * i] : dzt[1][2 * (i - 2)];
        const float gz1 = i < 2 ? dzt[0][2 * i + 1] : dzt[1][2 * (i - 2) + 1];
        if (feat_grad && si.valid && l < gd.levels)
          feat_grad[((int64_t)l * nqK + qj) * 16 + c] = make_float2(gz0 * delta[i], gz1 * delta[i]);
        dD = fmaf(gz0, dcoef[2 * i], fmaf(gz1, dcoef[2 * i + 1], dD));
      }
      dD += __shfl_xor(dD, 16, 64);
      dD += __shfl_xor(dD, 32, 64);
      if (g == 0 && si.valid && grad_depth) grad_depth[si.s] = si.has ? dD : 0.f;
    } else {
      // no unit for this wave in the last round: zero tiles add nothing
      for (int i = lane; i < UT::bytes / 4; i += 64) reinterpret_cast<uint32_t*>(T)[i] = 0u;
    }
    __syncthreads();
    // ---- this wave's share of the weight gradients over the round's NW units
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
      const unsigned char* U = tiles + u * UT::bytes;
      weight_grad_accum<BF, PAD, OT, CT3>(row_ptr(U, UT::oY3), row_ptr(U, UT::oX3 + 16 * CT3 * wave), accW3, lane);
      weight_grad_accum<BF, PAD, RT, MT>(row_ptr(U, UT::oY2 + 16 * RT * wave), row_ptr(U, UT::oX2), accW2, lane);
      weight_grad_accum<BF, PAD, RT, 2>(row_ptr(U, UT::oY1 + 16 * RT * wave), row_ptr(U, UT::oX1), accW1, lane);
    }
    __syncthreads();
  }
  // ---- add this wave's weight-gradient tiles to global memory
#pragma unroll
  for (int ot = 0; ot < OT; ++ot)
#pragma unroll
    for (int mi = 0; mi < CT3; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ot + 4 * g + r, col = 16 * (CT3 * wave + mi) + c;
        const float v = accW3[ot * CT3 + mi][r];
        if (g_w3 && row < LY::NOUT && v != 0.0f) unsafeAtomicAdd(&g_w3[row * HID + col], v);
      }
#pragma unroll
  for (int mo = 0; mo < RT; ++mo) {
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (RT * wave + mo) + 4 * g + r, col = 16 * mi + c;
        const float v = accW2[mo * MT + mi][r];
        if (g_w2 && v != 0.0f) unsafeAtomicAdd(&g_w2[row * HID + col], v);
      }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (RT * wave + mo) + 4 * g + r, col = 16 * mi + c;
        const float v = accW1[mo * 2 + mi][r];
        if (g_w1 && col < in_dim && v != 0.0f) unsafeAtomicAdd(&g_w1[row * in_dim + col], v);
      }
  }
}

// ------------------------------------------------------------------ hash scatter
// dL/dtheta for a table entry is the sum, over every sample and cell corner
// that hashes to it, of the corner's trilinear weight times the sample's
// feature gradient (FP32). It is formed level by level in two kernels that
// use no floating-point global atomics.
//
// scatter_bin: one task is one level over a block of 4x4-pixel patches (all
// K slots). Each wave sorts its 128 samples by cell (unless no neighbouring
// samples share one) and sums runs of equal cells; every run files 8 corner
// records (entry, 2 values) under their buckets, fixed ranges of
// 2^bucket_log2 table entries. The block ranks its records per bucket with
// LDS counters, groups them by bucket in LDS and appends them to the
// workgroup's own slab of each bucket (slab cursors stay in LDS for the whole
// launch, so filing needs no global atomics); at the end the workgroup writes
// its (slab start, count) per bucket into the slab table.
//
// scatter_reduce: one workgroup per bucket walks the bucket's column of the
// slab table, sums the records into a dense LDS array and adds it to its
// range of the gradient table, which no other workgroup writes.
//
// Measured on this chip: LDS float atomics (ds_add_f32) retire about one lane
// every three clocks per CU, integer LDS atomics about ten lanes per clock and
// a compare-and-swap several, so the LDS float sums are compare-and-swap loops
// on the 64-bit feature pair and the counting uses integer atomics.
constexpr int kScatThreads = 256;
constexpr int kReduceThreads = 1024;
constexpr int kReduceMaxLog2 = 13;  // LDS pairs per bucket in scatter_reduce
constexpr int kUnitsPerRow = kScatUnits / (kScatThreads / 16);
static_assert(kUnitsPerRow * (kScatThreads / 16) == kScatUnits, "units per task must fill the rows evenly");
constexpr int kMaxCasRounds = 256;  // default bound of lds_add_pair's retries

__device__ __forceinline__ unsigned long long pair_plus(unsigned long long old, float a, float b) {
  const float lo = __uint_as_float((uint32_t)old) + a;
  const float hi = __uint_as_float((uint32_t)(old >> 32)) + b;
  return ((unsigned long long)__float_as_uint(hi) << 32) | __float_as_uint(lo);
}

// Adds (a, b) to the pair at p with a compare-and-swap loop; false if it lost
// `rounds` races in a row (the caller then adds to global memory).
__device__ __forceinline__ bool lds_add_pair(unsigned long long* p, float a, float b, int rounds) {
  unsigned long long old = *p;
#pragma unroll 1
  for (int r = 0; r < rounds; ++r) {
    const unsigned long long prev = atomicCAS(p, old, pair_plus(old, a, b));
    if (prev == old) return true;
    old = prev;
  }
  return false;
}

constexpr uint32_t kInactiveKey = 0x1FFFFFFu;  // above every 24-bit hash
constexpr int kBlockSamples = kScatUnits * 16;  // 512 samples per task
static_assert(kBlockSamples == 2 * kScatThreads, "two samples per thread");
static_assert(kBlockRecords == 8 * kBlockSamples, "8 corner records per sample");
constexpr int kScatStageBytes = kBlockRecords * (sizeof(uint32_t) + sizeof(float2));
static_assert(kScatStageBytes >= sizeof(float) * 9 * kBlockSamples, "sample stage must fit the record stage");
static_assert(kScatMaxBuckets % kScatThreads == 0, "bucket counts split evenly over the threads");

// Cross-lane moves without the LDS permute path where the pattern allows:
// DPP (quad_perm, row_ror, wave and row shifts, row broadcasts) and the
// swizzle unit. dpp<CTRL, ROW_MASK>(v): lanes whose source is out of range,
// or whose row is not in ROW_MASK, read 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u(uint32_t v) {
  if constexpr (ROW_MASK == 0xF) {
    // every row enabled: out-of-range lanes read 0 (bound_ctrl), no old value
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
  } else {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
  }
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
  return __uint_as_float(dpp_u<CTRL, ROW_MASK>(__float_as_uint(v)));
}
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRowRor8 = 0x128;   // rotate by 8 within 16 lanes = xor 8
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShl2 = 0x102;   // lane i reads lane i + 2 within its row of 16
constexpr int kDppRowShl8 = 0x108;   // lane i reads lane i + 8 within its row of 16
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i - 1
constexpr int kDppWaveShl1 = 0x130;  // lane i reads lane i + 1
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// v of lane (lane ^ X), X a power of two below 64.
template <int X>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (X == 1) {
    return dpp_u<kDppQuadXor1>(v);
  } else if constexpr (X == 2) {
    return dpp_u<kDppQuadXor2>(v);
  } else if constexpr (X == 4) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1F);
  } else if constexpr (X == 8) {
    return dpp_u<kDppRowRor8>(v);
  } else if constexpr (X == 16) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (16 << 10) | 0x1F);
  } else {
    return (uint32_t)__shfl_xor((int)v, X, 64);
  }
}

// One compare-exchange stage (K_, J) of a bitonic sort of distinct keys for
// the two positions p0 = 2 l + base, p0 + 1 held by this lane (l = lane),
// J <= 64: the partner of a position lives in this lane (J = 1) or in lane
// l ^ (J / 2). Ascending runs of length KK alternate with descending ones.
template <int KK, int J>
__device__ __forceinline__ void bitonic_stage_regs(uint32_t (&key)[2], int p0) {
  if constexpr (J == 1) {
    const bool asc = (p0 & KK) == 0;
    const uint32_t lo = min(key[0], key[1]), hi = max(key[0], key[1]);
    key[0] = asc ? lo : hi;
    key[1] = asc ? hi : lo;
  } else {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = p0 + e;
      const uint32_t ok = lane_xor<J / 2>(key[e]);
      // the lower position of a pair keeps the smaller key in an ascending run
      const bool keep_min = ((p & J) == 0) == ((p & KK) == 0);
      key[e] = keep_min ? min(key[e], ok) : max(key[e], ok);
    }
  }
}

template <int KK, int J>
__device__ __forceinline__ void bitonic_merge_regs(uint32_t (&key)[2], int p0) {
  bitonic_stage_regs<KK, J>(key, p0);
  if constexpr (J > 1) bitonic_merge_regs<KK, J / 2>(key, p0);
}

template <int KK>
__device__ __forceinline__ void bitonic_sort_regs(uint32_t (&key)[2], int p0) {
  bitonic_merge_regs<KK, KK / 2>(key, p0);
  if constexpr (KK < 128) bitonic_sort_regs<KK * 2>(key, p0);
}

// Inclusive segmented scan across the 64 lanes: on return v holds the sum of
// v over the lanes from the start of this lane's segment (the nearest lane
// at or before it with head set; lane 0 must have it) to this lane. A step
// that reaches further back than any lane's segment start adds nothing and
// is skipped (at fine levels almost every segment is a single lane).
template <int N>
__device__ __forceinline__ void segmented_scan(float (&v)[N], bool head) {
  const int lane = threadIdx.x & 63;
  const unsigned long long heads = __ballot(head) | 1ull;
  const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  const int d = lane - (63 - __clzll(upto));  // lanes back to the segment start
  uint32_t h = head ? 1u : 0u;
  // a step adds the shifted value times keep (0 at a segment head, else 1):
  // one multiply-add per value, the same sum as a select between v and
  // v + shifted (x * 1 + v rounds once, like x + v)
#define NX_SEG_STEP(CTRL, MASK, NEEDED)                          \
  if (__any(NEEDED)) {                                           \
    const uint32_t sh = dpp_u<CTRL, MASK>(h);                    \
    const float keep = h ? 0.0f : 1.0f;                          \
    _Pragma("unroll") for (int q = 0; q < N; ++q)                \
      v[q] = fmaf(dpp_f<CTRL, MASK>(v[q]), keep, v[q]);          \
    h |= sh;                                                     \
  }
  NX_SEG_STEP(kDppRowShr1, 0xF, d >= 1)
  NX_SEG_STEP(kDppRowShr1 + 1, 0xF, d >= 2)
  NX_SEG_STEP(kDppRowShr1 + 3, 0xF, d >= 4)
  NX_SEG_STEP(kDppRowShr1 + 7, 0xF, d >= 8)
  NX_SEG_STEP(kDppRowBcast15, 0xA, d > (lane & 15))
  NX_SEG_STEP(kDppRowBcast31, 0xC, d > (lane & 31))
#undef NX_SEG_STEP
}

// The camera of a block: with JOINT the cameras' descriptors are read from
// device memory, otherwise the single camera's descriptor is the kernel
// argument itself (no loads beyond the argument segment).
template <bool JOINT>
__device__ __forceinline__ const ScatterCam& scatter_cam(const ScatterCam& cam0, const ScatterCam* cams, int i) {
  if constexpr (JOINT) {
    return cams[i];
  } else {
    return cam0;
  }
}

template <bool JOINT>
__global__ __launch_bounds__(kScatThreads) void scatter_bin_kernel(
    ScatterCam cam0, const ScatterCam* __restrict__ cams, int n_cams, int64_t n_blocks, int K, int log2K, int level,
    float* __restrict__ g_table, int log2_size, int bucket_log2, uint32_t slab, int64_t n_rows,
    uint2* __restrict__ slab_table, uint16_t* __restrict__ rec_key, float2* __restrict__ rec_val) {
  // LDS: the per-sample stage (corner values, cells, sort keys) and, once
  // those are in registers, the block's records grouped by bucket share one
  // region; per-bucket counters follow it (dynamic size: 4 nb words).
  extern __shared__ __attribute__((aligned(16))) unsigned char scat_lds[];
  // [e.x, e.y, fx, fy, fz][sample]: feature gradient and position in the cell
  auto& sfeat = *reinterpret_cast<float(*)[5][kBlockSamples]>(scat_lds);
  auto& scell = *reinterpret_cast<int(*)[kBlockSamples][3]>(scat_lds + sizeof(float) * 5 * kBlockSamples);
  uint32_t* skey = reinterpret_cast<uint32_t*>(scat_lds + sizeof(float) * 8 * kBlockSamples);
  uint32_t* st_h = reinterpret_cast<uint32_t*>(scat_lds);                          // record: entry index
  float2* st_v = reinterpret_cast<float2*>(scat_lds + sizeof(uint32_t) * kBlockRecords);  // record: 2 values
  const int nb = 1 << (log2_size - bucket_log2);
  uint32_t* hist = reinterpret_cast<uint32_t*>(scat_lds + kScatStageBytes);  // count, then local offset
  // per bucket: (record slot of local position 0, first local position that
  // no longer fits the slab)
  uint2* gslot = reinterpret_cast<uint2*>(hist + nb);
  uint32_t* wcur = hist + 3 * nb;  // records this workgroup has filed per bucket
  __shared__ uint32_t wsum[kScatThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = lane & 15;
  const int row = threadIdx.x >> 4;
  const uint32_t mask = (1u << log2_size) - 1u;
  const uint32_t emask = (1u << bucket_log2) - 1u;
  float* g_level = g_table + 2 * ((size_t)level << log2_size);
  const int p0 = 128 * wave + 2 * lane;  // sorted positions p0, p0 + 1 belong to this lane
  // Consecutive workgroup ids go to different XCDs; renumber so that each XCD
  // walks neighbouring blocks.
  const int G = gridDim.x;
  const int wg = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const size_t slab_base = (size_t)wg * nb * slab;  // this workgroup's slab of bucket 0
  const uint32_t slab_base32 = (uint32_t)slab_base;  // the launch keeps every slot below 2^32
  for (int i = threadIdx.x; i < nb; i += kScatThreads) wcur[i] = 0u;
  int cam = 0;  // blocks ascend, so the camera only moves forward
  for (int64_t blk = wg; blk < n_blocks; blk += G) {
    if constexpr (JOINT) {
      while (cam + 1 < n_cams && cams[cam + 1].blk0 <= blk) ++cam;
    }
    const ScatterCam& sc = scatter_cam<JOINT>(cam0, cams, cam);
    const GridDev& gd = sc.gd;
    const GridLevel L = gd.lv[level];
    const float* __restrict__ depths = sc.depths;
    const float2* __restrict__ feat_grad = sc.feat_grad;
    const int bw = sc.bw, bh = sc.bh, nbx = sc.nbx;
    const int log2bw = __builtin_ctz((unsigned)bw);  // bw is a power of two
    const int npx = (gd.width + 3) >> 2, npy = (gd.height + 3) >> 2;
    const int64_t nqK = (int64_t)npx * npy * K;
    const float2* __restrict__ fg_level = feat_grad + (size_t)level * (size_t)nqK * 16;
    const int64_t lb = blk - sc.blk0;
    for (int i = threadIdx.x; i < nb; i += kScatThreads) hist[i] = 0u;
    const int bx = (int)(lb % nbx), by = (int)(lb / nbx);
    // 1. per sample: cell, position in it, feature gradient and sort key
#pragma unroll
    for (int it = 0; it < kUnitsPerRow; ++it) {
      const int u = row + it * (kScatThreads / 16);
      const int smp = u * 16 + c;
      const int pb = u >> log2K, j = u & (K - 1);
      const int qx = bx * bw + (pb & (bw - 1)), qy = by * bh + (pb >> log2bw);
      const bool in = qx < npx && qy < npy;
      const SampleInfo si = sample_ray_xy(gd, K, in ? qx : 0, in ? qy : 0, j, c, depths);
      float2 e = make_float2(0.f, 0.f);
      // the level's rows start at fg_level; a unit's index within the level
      // (patches x K, below 2^28) fits 32 bits
      if (in && si.valid) e = fg_level[(size_t)((uint32_t)(qy * npx + qx) * (uint32_t)K + (uint32_t)j) * 16 + c];
      const bool act = in & si.valid & ((e.x != 0.f) | (e.y != 0.f));
      const LevelGeom lg = level_geom(L, si);
      sfeat[0][smp] = act ? e.x : 0.f;
      sfeat[1][smp] = act ? e.y : 0.f;
      sfeat[2][smp] = lg.frx;
      sfeat[3][smp] = lg.fry;
      sfeat[4][smp] = lg.frz;
      scell[smp][0] = lg.cx;
      scell[smp][1] = lg.cy;
      scell[smp][2] = lg.cz;
      // sort key: the low 8 bits of the three cell coordinates (24 bits, no
      // multiplies; two cells of one wave share them only if they differ by
      // multiples of 256 on all three axes) above the sample's index within
      // its wave's 128; inactive samples get a larger prefix, sort last and
      // form no records. Two cells that share the 24 bits only form two
      // segments, as the segments compare the cells themselves.
      const uint32_t ck = ((uint32_t)lg.cx & 0xFFu) | (((uint32_t)lg.cy & 0xFFu) << 8) | (((uint32_t)lg.cz & 0xFFu) << 16);
      const uint32_t hk = act ? ck : kInactiveKey;
      skey[smp] = (hk << 7) | (uint32_t)(smp & 127);
    }
    __syncthreads();
    // 2. bitonic sort of (key, sample) over each wave's 128 samples (the
    // wave's two patches, all slots); equal cells in different waves stay
    // separate records, which only costs a few duplicates at coarse levels.
    // In pixel order a lane holds two horizontally adjacent pixels of one
    // slot, lane + 2 the pixels below them and lane + 8 the same pixels at the
    // next slot. When no such pair shares a cell (fine levels: a pixel spans
    // a cell or more), sorting would gather next to nothing, and the wave
    // keeps pixel order: runs of equal cells are still summed where they are
    // adjacent, and the others file separate records, which the reduction
    // adds up like any others.
    uint32_t key[2] = {skey[p0], skey[p0 + 1]};
    {
      const uint32_t h0 = key[0] >> 7, h1 = key[1] >> 7;
      const uint32_t below = dpp_u<kDppRowShl2>(h0), next_slot = dpp_u<kDppRowShl8>(h0);
      const bool live0 = h0 != kInactiveKey;
      // bitwise, not short-circuit (each && or || would be a branch on the execution mask)
      const bool shared =
          live0 & ((h0 == h1) | (((lane & 15) < 14) & (h0 == below)) | (((lane & 15) < 8) & (h0 == next_slot)));
      if (__any(shared)) bitonic_sort_regs<2>(key, p0);
    }
    // 3. segments of equal cells along the sorted order, summed within each wave
    bool live[2];
    int cx[2], cy[2], cz[2];
    float a[2][16];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int sm = 128 * wave + (int)(key[e] & 127u);
      live[e] = (key[e] >> 7) != kInactiveKey;
      cx[e] = scell[sm][0];
      cy[e] = scell[sm][1];
      cz[e] = scell[sm][2];
      // the 16 corner contributions: trilinear weight x feature gradient
      LevelGeom fr;
      fr.frx = sfeat[2][sm];
      fr.fry = sfeat[3][sm];
      fr.frz = sfeat[4][sm];
      const float ex = sfeat[0][sm], ey = sfeat[1][sm];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const float w = corner_weight(fr, b);
        a[e][2 * b] = w * ex;
        a[e][2 * b + 1] = w * ey;
      }
    }
    // element 1 continues element 0's segment?
    const bool same01 = (live[0] == live[1]) & (cx[0] == cx[1]) & (cy[0] == cy[1]) & (cz[0] == cz[1]);
    // previous lane's last element continues into this lane's element 0?
    const int pcx = (int)dpp_u<kDppWaveShr1>((uint32_t)cx[1]), pcy = (int)dpp_u<kDppWaveShr1>((uint32_t)cy[1]);
    const int pcz = (int)dpp_u<kDppWaveShr1>((uint32_t)cz[1]);
    const bool plive = dpp_u<kDppWaveShr1>(live[1] ? 1u : 0u) != 0u;
    const bool cont0 = (lane > 0) & (plive == live[0]) & (pcx == cx[0]) & (pcy == cy[0]) & (pcz == cz[0]);
    // next lane's element 0 continues element 1's segment?
    const bool next_cont = dpp_u<kDppWaveShl1>(cont0 ? 1u : 0u) != 0u;
    const bool tail1 = lane == 63 || !next_cont;
    const bool tail0 = !same01;
    // 4. records: a segment tail emits its cell's 8 corners (a record whose
    // two values are zero is filed like any other). Which records exist is
    // known before their values, so they are counted first: the count's old
    // value is the record's rank among the block's records of its bucket.
    const bool emit[2] = {(bool)(tail0 & live[0]), (bool)(tail1 & live[1])};
    uint32_t rh[2][8], rank[2][8];  // rank: only where emit
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const uint32_t hx0 = map_positive(cx[e]), hx1 = map_positive(cx[e] + 1);
      const uint32_t hy0 = map_positive(cy[e]) * kPrime1, hy1 = map_positive(cy[e] + 1) * kPrime1;
      const uint32_t hz0 = map_positive(cz[e]) * kPrime2, hz1 = map_positive(cz[e] + 1) * kPrime2;
#pragma unroll
      for (int b = 0; b < 8; ++b) rh[e][b] = ((b & 1 ? hx1 : hx0) ^ (b & 2 ? hy1 : hy0) ^ (b & 4 ? hz1 : hz0)) & mask;
      if (emit[e]) {  // one branch for the element's 8 counts
#pragma unroll
        for (int b = 0; b < 8; ++b) rank[e][b] = atomicAdd(&hist[rh[e][b] >> bucket_log2], 1u);
      }
    }
    __syncthreads();
    // 5. local offsets of the buckets (exclusive scan of the counts) and the
    // slots this block takes in the workgroup's slabs
    uint32_t n_rec = 0;
    {
      const int per = nb > kScatThreads ? nb / kScatThreads : 1;
      const int b0 = threadIdx.x * per;
      uint32_t cnt[kScatMaxBuckets / kScatThreads];
      uint32_t run = 0;
#pragma unroll
      for (int i = 0; i < kScatMaxBuckets / kScatThreads; ++i) {
        cnt[i] = (i < per && b0 + i < nb) ? hist[b0 + i] : 0u;
        run += cnt[i];
      }
      uint32_t incl = run;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
      }
      if (lane == 63) wsum[wave] = incl;
      __syncthreads();
      uint32_t before = 0, total = 0;
#pragma unroll
      for (int w = 0; w < kScatThreads / 64; ++w) {
        const uint32_t t = wsum[w];
        before += w < wave ? t : 0u;
        total += t;
      }
      uint32_t off = before + incl - run;
#pragma unroll
      for (int i = 0; i < kScatMaxBuckets / kScatThreads; ++i) {
        if (i < per && b0 + i < nb) {
          const uint32_t used = wcur[b0 + i];
          // a record at local position i goes to slot i + used - off of the
          // bucket's slab, if that is below slab
          gslot[b0 + i] = make_uint2(slab_base32 + (uint32_t)(b0 + i) * slab + used - off,
                                     (uint32_t)((int)off + (int)slab - (int)used));
          wcur[b0 + i] = used + cnt[i];
          hist[b0 + i] = off;  // from here on: the bucket's local offset
          off += cnt[i];
        }
      }
      n_rec = total;
      __syncthreads();
    }
    // 6. values: element 1's lane value is the sum of its segment within this
    // lane (head: that segment starts in this lane), summed across lanes;
    // element 0 takes the carry from earlier lanes of its segment
    float s1[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) s1[v] = same01 ? a[0][v] + a[1][v] : a[1][v];
    segmented_scan<16>(s1, !(same01 && cont0));
    float carry[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) carry[v] = dpp_f<kDppWaveShr1>(s1[v]);
    // records into LDS, grouped by bucket (local offset + rank)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (emit[e]) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const float v0 = e == 0 ? (cont0 ? carry[2 * b] + a[0][2 * b] : a[0][2 * b]) : s1[2 * b];
          const float v1 = e == 0 ? (cont0 ? carry[2 * b + 1] + a[0][2 * b + 1] : a[0][2 * b + 1]) : s1[2 * b + 1];
          const uint32_t at = hist[rh[e][b] >> bucket_log2] + rank[e][b];
          st_h[at] = rh[e][b];
          st_v[at] = make_float2(v0, v1);
        }
      }
    }
    __syncthreads();
    // 7. consecutive records of a bucket go to consecutive global slots (four
    // records per thread in flight)
    for (uint32_t i0 = threadIdx.x; i0 < n_rec; i0 += 4 * kScatThreads) {
      uint32_t h[4];
      float2 v[4];
      uint2 gs[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * kScatThreads;
        h[u] = i < n_rec ? st_h[i] : 0u;
        v[u] = i < n_rec ? st_v[i] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) gs[u] = gslot[h[u] >> bucket_log2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * kScatThreads;
        if (i >= n_rec) continue;
        if ((int)i < (int)gs[u].y) {
          const uint32_t at = gs[u].x + i;
          rec_key[at] = (uint16_t)(h[u] & emask);
          rec_val[at] = v[u];
        } else {  // slab full: add straight into the table
          unsafeAtomicAdd(&g_level[2 * (size_t)h[u]], v[u].x);
          unsafeAtomicAdd(&g_level[2 * (size_t)h[u] + 1], v[u].y);
        }
      }
    }
    __syncthreads();
  }
  // 8. the workgroup's slab of every bucket: start and records in it
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kScatThreads) {
    const uint32_t n = wcur[i];
    slab_table[(size_t)i * n_rows + wg] = make_uint2((uint32_t)(slab_base + (size_t)i * slab), n < slab ? n : slab);
  }
}

// Sorts (key, a, b) across the 64 lanes by key, ascending (keys distinct or
// not; equal keys end up adjacent).
__device__ __forceinline__ void wave_sort_by_key(uint32_t& key, float& a, float& b) {
  const int lane = threadIdx.x & 63;
#define NX_WS_STAGE(KK, J)                                                          \
  {                                                                                 \
    const uint32_t ok = lane_xor<J>(key);                                           \
    const float oa = __uint_as_float(lane_xor<J>(__float_as_uint(a)));              \
    const float ob = __uint_as_float(lane_xor<J>(__float_as_uint(b)));              \
    const bool keep_min = ((lane & J) == 0) == ((lane & KK) == 0);                  \
    const bool take = keep_min ? ok < key : ok > key;                               \
    key = take ? ok : key;                                                          \
    a = take ? oa : a;                                                              \
    b = take ? ob : b;                                                              \
  }
  NX_WS_STAGE(2, 1)
  NX_WS_STAGE(4, 2) NX_WS_STAGE(4, 1)
  NX_WS_STAGE(8, 4) NX_WS_STAGE(8, 2) NX_WS_STAGE(8, 1)
  NX_WS_STAGE(16, 8) NX_WS_STAGE(16, 4) NX_WS_STAGE(16, 2) NX_WS_STAGE(16, 1)
  NX_WS_STAGE(32, 16) NX_WS_STAGE(32, 8) NX_WS_STAGE(32, 4) NX_WS_STAGE(32, 2) NX_WS_STAGE(32, 1)
  NX_WS_STAGE(64, 32) NX_WS_STAGE(64, 16) NX_WS_STAGE(64, 8) NX_WS_STAGE(64, 4) NX_WS_STAGE(64, 2)
  NX_WS_STAGE(64, 1)
#undef NX_WS_STAGE
}

template <int KR>
__global__ __launch_bounds__(kReduceThreads) void scatter_reduce_kernel(int bucket_log2, int coarse, int cas_rounds,
                                                                       int64_t n_rows,
                                                                       const uint2* __restrict__ slab_table,
                                                                       const uint16_t* __restrict__ rec_key,
                                                                       const float2* __restrict__ rec_val,
                                                                       float* __restrict__ g_level) {
  // the bucket's entries as (feature 0, feature 1) float pairs; sized to the
  // bucket at launch, so that binning workgroups of the next level still fit
  // next to it on the CU
  extern __shared__ unsigned long long acc[];
  const int b = blockIdx.x;
  const int n_e = 1 << bucket_log2;
  for (int i = threadIdx.x; i < n_e; i += kReduceThreads) acc[i] = 0ull;
  __syncthreads();
  float2* out = reinterpret_cast<float2*>(g_level) + ((size_t)b << bucket_log2);
  const uint2* col = slab_table + (size_t)b * n_rows;
  // 16-lane groups walk the slabs (one row each, 64 rows at a time)
  const int grp = threadIdx.x >> 4, c = threadIdx.x & 15;
  constexpr int kGroups = kReduceThreads / 16;
  if (coarse) {
    // Coarse level: few entries take many records each, so equal keys meet
    // in one instruction; each wave first sorts its 64 records by key and
    // sums runs of equal keys, and only the last record of a run goes to LDS.
    const int lane = threadIdx.x & 63;
    for (int64_t r0 = grp - (grp & 3); r0 < n_rows; r0 += kGroups) {  // uniform per wave
      const int64_t r = r0 + (grp & 3);
      const uint2 sl = r < n_rows ? col[r] : make_uint2(0u, 0u);
      for (uint32_t i0 = 0; __any(i0 < sl.y); i0 += 16) {
        const uint32_t i = i0 + c;
        const bool ok = i < sl.y;
        uint32_t key = ok ? (uint32_t)rec_key[sl.x + i] : 0xFFFFFFFFu;
        float2 v = ok ? rec_val[sl.x + i] : make_float2(0.f, 0.f);
        wave_sort_by_key(key, v.x, v.y);
        const uint32_t prev = dpp_u<kDppWaveShr1>(key), next = dpp_u<kDppWaveShl1>(key);
        float s2[2] = {v.x, v.y};
        segmented_scan<2>(s2, lane == 0 || prev != key);
        if (key != 0xFFFFFFFFu && (lane == 63 || next != key) && !lds_add_pair(&acc[key], s2[0], s2[1], cas_rounds)) {
          unsafeAtomicAdd(&out[key].x, s2[0]);
          unsafeAtomicAdd(&out[key].y, s2[1]);
        }
      }
    }
  } else {
    // Fine level: a group keeps up to kU records of each of KR rows in
    // flight. Where a slab row holds only a few dozen records (a few blocks
    // per binning workgroup), walking one row at a time would wait on two
    // dependent memory reads (the row's slab entry, then its records) per few
    // dozen records, so KR = 4; longer rows keep a group busy with KR = 1.
    constexpr int kU = 4, kR = KR;
    for (int64_t r0 = grp; r0 < n_rows; r0 += (int64_t)kGroups * kR) {
      uint2 sl[kR];
      uint32_t most = 0;
#pragma unroll
      for (int q = 0; q < kR; ++q) {
        const int64_t r = r0 + (int64_t)q * kGroups;
        sl[q] = r < n_rows ? col[r] : make_uint2(0u, 0u);
        most = max(most, sl[q].y);
      }
      for (uint32_t i0 = c; i0 < most; i0 += 16 * kU) {
        uint32_t k[kR][kU];
        float2 v[kR][kU];
#pragma unroll
        for (int q = 0; q < kR; ++q)
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + 16 * u;
            const bool ok = i < sl[q].y;
            k[q][u] = ok ? (uint32_t)rec_key[sl[q].x + i] : 0u;
            v[q][u] = ok ? rec_val[sl[q].x + i] : make_float2(0.f, 0.f);
          }
#pragma unroll
        for (int q = 0; q < kR; ++q)
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            if (i0 + 16 * u < sl[q].y && !lds_add_pair(&acc[k[q][u]], v[q][u].x, v[q][u].y, cas_rounds)) {
              unsafeAtomicAdd(&out[k[q][u]].x, v[q][u].x);
              unsafeAtomicAdd(&out[k[q][u]].y, v[q][u].y);
            }
          }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_e; i += kReduceThreads) {
    const unsigned long long pv = acc[i];
    if (pv != 0ull) {
      float2 o = out[i];
      o.x += __uint_as_float((uint32_t)pv);
      o.y += __uint_as_float((uint32_t)(pv >> 32));
      out[i] = o;
    }
  }
}

__global__ void copy_plain_kernel(const float* plain, float* image, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) image[i] = plain[i];
}

int ilog2(int k) {
  int r = 0;
  while ((1 << r) < k) ++r;
  return r;
}

template <int TDT, bool BF, int HID, bool SH>
hipError_t fwd_inst(const GridDev& gd, const void* table, const MlpDev& mlp, int K, int64_t n_samples,
                    const int32_t* ids, const float* depths, const float* weights, const float* plain, float* tex,
                    float* image, int32_t* cells, uint32_t* masks, float* feats, hipStream_t s) {
  const int64_t n_q = n_patches(gd);
  int64_t grid = (n_q + kWaves - 1) / kWaves;
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((texture_forward_kernel<TDT, BF, HID, SH>), dim3((unsigned)grid), dim3(kTexThreads), 0, s, gd,
                     table, mlp.w[0], mlp.w[1], mlp.w[2], mlp.in_dim, K, ilog2(K), n_samples, ids, depths, weights,
                     plain, tex, image, cells, masks, feats);
  return hipGetLastError();
}

template <int TDT, bool BF, int HID, bool SH>
hipError_t bwd_inst(const GridDev& gd, const void* table, const MlpDev& mlp, int K, int64_t n_samples,
                    const int32_t* ids, const float* depths, const float* weights, const float* grad_image,
                    const float* grad_tex, float2* feat_grad, float* g0, float* g1, float* g2, float* grad_depth,
                    unsigned char* wop, hipStream_t s) {
  // operand slots in LDS for the BF16 hidden-64 RGB form; the others read them
  // from the workspace (L2-resident), leaving LDS to the activation tiles
  constexpr bool kWlds = HID <= 64 && BF && !SH;
  constexpr int NW = bwd_waves(BF, HID);
  const int64_t n_q = n_patches(gd) * K;
  int64_t grid = (n_q + NW - 1) / NW;
  // about two workgroups' worth per resident slot (two per CU with 4 waves,
  // one with 8)
  const int64_t max_grid = NW == 8 ? 512 : 1024;
  if (grid > max_grid) grid = max_grid;
  if (grid < 1) grid = 1;
  if constexpr (!kWlds) {
    hipLaunchKernelGGL((stage_weight_operands_kernel<BF, HID, SH>), dim3(64), dim3(256), 0, s, wop, mlp.w[0],
                       mlp.w[1], mlp.w[2], mlp.in_dim);
  }
  hipLaunchKernelGGL((texture_backward_kernel<TDT, BF, HID, SH, kWlds>), dim3((unsigned)grid), dim3(64 * NW), 0,
                     s, gd, table, mlp.w[0], mlp.w[1], mlp.w[2], wop, mlp.in_dim, K, ilog2(K), n_samples, ids, depths,
                     weights, grad_image, grad_tex, feat_grad, g0, g1, g2, grad_depth);
  return hipGetLastError();
}

// Arguments of one texturing-pass launch, forwarded to the instantiation the
// storage types, hidden width and head select.
struct TexArgs {
  GridDev gd;
  const void* table;
  MlpDev mlp;
  int K;
  int64_t n;
  const int32_t* ids;
  const float *depths, *weights;
  // forward
  const float* plain;
  float *tex, *image;
  int32_t* cells;
  uint32_t* masks;
  float* feats;
  // backward
  const float *grad_image, *grad_tex;
  float2* feat_grad;
  float *g0, *g1, *g2, *grad_depth;
  unsigned char* wop;
};

template <int TDT, bool BF, int HID, bool SH>
hipError_t run_tex(bool backward, const TexArgs& a, hipStream_t s) {
  if (backward)
    return bwd_inst<TDT, BF, HID, SH>(a.gd, a.table, a.mlp, a.K, a.n, a.ids, a.depths, a.weights, a.grad_image,
                                      a.grad_tex, a.feat_grad, a.g0, a.g1, a.g2, a.grad_depth, a.wop, s);
  return fwd_inst<TDT, BF, HID, SH>(a.gd, a.table, a.mlp, a.K, a.n, a.ids, a.depths, a.weights, a.plain, a.tex,
                                    a.image, a.cells, a.masks, a.feats, s);
}

template <bool BF, int HID, bool SH>
hipError_t by_table(int tdt, bool backward, const TexArgs& a, hipStream_t s) {
  switch (tdt) {
    case NX_F32: return run_tex<NX_F32, BF, HID, SH>(backward, a, s);
    case NX_F16: return run_tex<NX_F16, BF, HID, SH>(backward, a, s);
    case NX_BF16: return run_tex<NX_BF16, BF, HID, SH>(backward, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool SH>
hipError_t by_mlp(int tdt, int mlp_dtype, bool backward, const TexArgs& a, hipStream_t s) {
  const bool bf = mlp_dtype == NX_BF16;
  if (a.mlp.hidden == 64)
    return bf ? by_table<true, 64, SH>(tdt, backward, a, s) : by_table<false, 64, SH>(tdt, backward, a, s);
  if (a.mlp.hidden == 128)
    return bf ? by_table<true, 128, SH>(tdt, backward, a, s) : by_table<false, 128, SH>(tdt, backward, a, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_texture_forward(int K, int feat_dtype, int mlp_dtype, int sh, const GridDev& grid,
                                  const void* table, const MlpDev& mlp, const int32_t* ids, const float* depths,
                                  const float* weights, const float* plain, float* tex, float* image, int32_t* cells,
                                  uint32_t* masks, float* feats, hipStream_t s) {
  const int64_t P = (int64_t)grid.width * grid.height;
  if (K == 0) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_plain_kernel, dim3((unsigned)((3 * P + 255) / 256)), dim3(256), 0, s, plain, image, 3 * P);
    return hipGetLastError();
  }
  const int64_t n = P * K;
  if (n == 0) return hipSuccess;
  TexArgs a{};
  a.gd = grid;
  a.table = table;
  a.mlp = mlp;
  a.K = K;
  a.n = n;
  a.ids = ids;
  a.depths = depths;
  a.weights = weights;
  a.plain = plain;
  a.tex = tex;
  a.image = image;
  a.cells = cells;
  a.masks = masks;
  a.feats = feats;
  return sh ? by_mlp<true>(feat_dtype, mlp_dtype, false, a, s) : by_mlp<false>(feat_dtype, mlp_dtype, false, a, s);
}

hipError_t launch_texture_backward(int K, int feat_dtype, int mlp_dtype, int sh, const GridDev& grid,
                                   const void* table, const MlpDev& mlp, const int32_t* ids, const float* depths,
                                   const float* weights, const float* grad_image, const float* grad_tex,
                                   float2* feat_grad, float* g_mlp0, float* g_mlp1, float* g_mlp2, float* grad_depth,
                                   unsigned char* weight_ops, hipStream_t s) {
  const int64_t P = (int64_t)grid.width * grid.height;
  if (K == 0) return hipSuccess;
  const int64_t n = P * K;
  if (n == 0) return hipSuccess;
  TexArgs a{};
  a.gd = grid;
  a.table = table;
  a.mlp = mlp;
  a.K = K;
  a.n = n;
  a.ids = ids;
  a.depths = depths;
  a.weights = weights;
  a.grad_image = grad_image;
  a.grad_tex = grad_tex;
  a.feat_grad = feat_grad;
  a.g0 = g_mlp0;
  a.g1 = g_mlp1;
  a.g2 = g_mlp2;
  a.grad_depth = grad_depth;
  a.wop = weight_ops;
  return sh ? by_mlp<true>(feat_dtype, mlp_dtype, true, a, s) : by_mlp<false>(feat_dtype, mlp_dtype, true, a, s);
}

namespace {
struct ScatterLaunch {
  int bl, nb;  // log2 entries per bucket, buckets
};
bool scatter_launch(const GridDev& grid, ScatterLaunch* o) {
  o->bl = scatter_bucket_log2(grid.log2_size);
  o->nb = scatter_buckets(grid.log2_size);
  return o->bl <= kReduceMaxLog2 && o->nb <= kScatMaxBuckets;
}

__global__ void write_scatter_cam_kernel(ScatterCam cam, ScatterCam* dst) {
  // a plain copy of the argument, one dword per lane
  static_assert(sizeof(ScatterCam) % 4 == 0, "copied in dwords");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&cam);
  uint32_t* out = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(ScatterCam) / 4); i += blockDim.x) out[i] = src[i];
}
}  // namespace

hipError_t launch_write_scatter_cam(const ScatterCam& cam, ScatterCam* dst, hipStream_t s) {
  hipLaunchKernelGGL(write_scatter_cam_kernel, dim3(1), dim3(256), 0, s, cam, dst);
  return hipGetLastError();
}

hipError_t launch_hash_scatter_bin(int K, const ScatterCam& cam0, const ScatterCam* cams, int n_cams, int64_t n_blocks,
                                   const GridDev& grid0, int level, float* g_table, int64_t n_rows, uint2* slab_table,
                                   uint16_t* rec_key, float2* rec_val, int64_t slab_cap, hipStream_t s) {
  if (K == 0 || n_blocks <= 0 || n_cams <= 0 || level < 0 || level >= grid0.levels) return hipSuccess;
  ScatterLaunch sl;
  if (!scatter_launch(grid0, &sl)) return hipErrorInvalidValue;
  const ScatterSlabs sb = scatter_slabs_blocks(n_blocks, sl.nb);
  if (sb.wgs > n_rows || sb.wgs * sl.nb * sb.slab > 0xFFFFFFFFll) return hipErrorInvalidValue;
  const size_t lds = kScatStageBytes + 4 * sizeof(uint32_t) * sl.nb;
  // a smaller slab (diagnostics) stays inside the records laid out for the full one
  const int64_t slab = slab_cap > 0 && slab_cap < sb.slab ? slab_cap : sb.slab;
  if (n_cams == 1) {
    hipLaunchKernelGGL(scatter_bin_kernel<false>, dim3((unsigned)sb.wgs), dim3(kScatThreads), lds, s, cam0, cams,
                       n_cams, n_blocks, K, ilog2(K), level, g_table, grid0.log2_size, sl.bl, (uint32_t)slab, n_rows,
                       slab_table, rec_key, rec_val);
  } else {
    if (!cams) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scatter_bin_kernel<true>, dim3((unsigned)sb.wgs), dim3(kScatThreads), lds, s, cam0, cams, n_cams,
                       n_blocks, K, ilog2(K), level, g_table, grid0.log2_size, sl.bl, (uint32_t)slab, n_rows,
                       slab_table, rec_key, rec_val);
  }
  return hipGetLastError();
}

hipError_t launch_hash_scatter_reduce(const GridDev& grid, int level, float* g_table, int64_t n_rows,
                                      int64_t n_blocks, const uint2* slab_table, const uint16_t* rec_key,
                                      const float2* rec_val, int cas_rounds, hipStream_t s) {
  if (level < 0 || level >= grid.levels || n_rows <= 0) return hipSuccess;
  ScatterLaunch sl;
  if (!scatter_launch(grid, &sl)) return hipErrorInvalidValue;
  // a level whose lattice has fewer than 2^16 corners (s_l + 2)^3 spreads its
  // records over at most that many entries
  const float corners = (grid.lv[level].scale + 2.0f) * (grid.lv[level].scale + 2.0f) * (grid.lv[level].scale + 2.0f);
  const int coarse = corners < 65536.0f ? 1 : 0;
  const size_t lds = sizeof(unsigned long long) << sl.bl;
  const int rounds = cas_rounds > 0 ? cas_rounds : kMaxCasRounds;
  float* g_level = g_table + 2 * ((size_t)level << grid.log2_size);
  // measured: four rows at once pays at 8 blocks per binning workgroup (one
  // 1080p camera) and costs at about 60 (sixteen cameras)
  if (n_blocks <= 16 * n_rows) {
    hipLaunchKernelGGL(scatter_reduce_kernel<4>, dim3((unsigned)sl.nb), dim3(kReduceThreads), lds, s, sl.bl, coarse,
                       rounds, n_rows, slab_table, rec_key, rec_val, g_level);
  } else {
    hipLaunchKernelGGL(scatter_reduce_kernel<1>, dim3((unsigned)sl.nb), dim3(kReduceThreads), lds, s, sl.bl, coarse,
                       rounds, n_rows, slab_table, rec_key, rec_val, g_level);
  }
  return hipGetLastError();
}

}  // namespace nx
