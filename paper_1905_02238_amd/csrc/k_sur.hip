// k_sur.hip -- the learned surrogate: a small conv net that predicts a pose's
// mutual information from the occupancy patch around it, trained on labels the
// exact FSMI path produces, and a ranking path whose top-k candidates are always
// re-scored by exact FSMI.
//
// Network (per pose): 128 x 128 patch of o around the pose (cells outside the
// map read 0.5) -> five 3x3 convolutions, stride 2, padding 1, ReLU
// (1->32->64->64->128->128 channels; 128 -> 64 -> 32 -> 16 -> 8 -> 4 pixels) ->
// global average pool -> FC 128->256 -> ReLU -> FC 256->1.  The regression
// target of a label is exp((MI - mean)/scale), standardised (sur_target); the
// loss is the batch-mean squared error, and predictions are mapped back to
// nats.
//
// Layout: activations NHWC in BF16, conv weights [co][tap][ci] (and a copy
// [tap][ci][co] for the input-gradient pass) in BF16, FP32 master weights,
// FP32 gradients and Adam moments.  The convolutions are implicit GEMMs on
// the gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; the first layer gathers its input straight from the map.
// Weight-gradient reductions are split over fixed pixel ranges and summed in a
// fixed order, so training is deterministic.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "fsmi_dev.h"
#include "fsmi_internal.h"

namespace fsmi {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Parameter layout (FP32 master, flat)
// ---------------------------------------------------------------------------
struct LayerDims { int cin, cout, hin; };
constexpr LayerDims kL[5] = {{1, 32, 128}, {32, 64, 64}, {64, 64, 32}, {64, 128, 16}, {128, 128, 8}};
constexpr int kPatch = 128, kFeat = 128, kHid = 256;

constexpr int w_size(int l) { return kL[l].cout * 9 * kL[l].cin; }
constexpr int w_off(int l) {  // FP32 master offset of conv l's weights
  int o = 0;
  for (int i = 0; i < l; ++i) o += w_size(i) + kL[i].cout;
  return o;
}
constexpr int b_off(int l) { return w_off(l) + w_size(l); }
constexpr int wbf_off(int l) {  // BF16 weight offset
  int o = 0;
  for (int i = 0; i < l; ++i) o += w_size(i);
  return o;
}
constexpr int kWbfTotal = wbf_off(5);
constexpr int kF1 = w_off(5);             // FC1 weights [256][128]
constexpr int kC1 = kF1 + kHid * kFeat;   // FC1 bias [256]
constexpr int kF2 = kC1 + kHid;           // FC2 weights [256]
constexpr int kC2 = kF2 + kHid;           // FC2 bias
constexpr int kNumParams = kC2 + 1;
static_assert(kNumParams == 310465, "parameter count");

int64_t sur_num_params() { return kNumParams; }

// ---------------------------------------------------------------------------
// MFMA fragment helpers (v_mfma_f32_16x16x32_bf16, wave64):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + 0..7]
//   B (32 x 16): lane l holds B[8 (l / 16) + 0..7][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + 0..3][l % 16]
// ---------------------------------------------------------------------------
FSMI_DEV floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// v_mfma_f32_16x16x16_bf16: as above with K = 16, lane l holding A[l % 16][4 (l / 16) + 0..3]
// and B[4 (l / 16) + 0..3][l % 16].
typedef short shortx4 __attribute__((ext_vector_type(4)));
FSMI_DEV floatx4 mfma16(bf16x4 a, bf16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(shortx4, a),
                                                   __builtin_bit_cast(shortx4, b), c, 0, 0, 0);
}
FSMI_DEV bf16x8 load8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
FSMI_DEV bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int q = 0; q < 8; ++q) z[q] = (bf16)0.0f;
  return z;
}

// Input of the first layer: patch pixel (iy, ix) of pose b is 0 outside the
// padded patch (iy or ix outside [0, 128)), else the map resampled at the
// pose's continuous position: with (u, v) = (x / s, y / s) the pose in block
// units, the bilinear interpolation of the map's blocks (block k centred at
// k + 1/2, 0.5 outside the map) at (u - 64 + ix + 1/2, v - 64 + iy + 1/2),
// i.e. blocks (floor(u) - 64 + ix + {0, 1}, floor(v) - 64 + iy + {0, 1})
// weighted by the pose's fraction (u - floor(u), v - floor(v)) inside its
// block, the same for every pixel.  So the patch moves with the pose's
// sub-block position.  With cell stride s > 1, `map` is the map of s x s
// block means; s = 1 reads the map itself.
// A pose's block (bx, by) and its fraction (fx, fy) inside that block: what
// every tile of its patch needs from the pose, computed once per pose of a
// batch (k_patch_origin) instead of once per tile (four FP64 divisions).
struct PatchOrigin {
  int bx, by;
  float fx, fy;
};

struct PatchSrc {
  const float* map;
  int64_t X, Y;          // dims of `map`
  const double* poses;   // [n][4]
  int s;                 // cell stride
  const PatchOrigin* org = nullptr;   // per pose of the batch (k_patch_origin)
  // floor(floor(v) / s), exact in FP64 for |v| < 2^53 (a quotient of
  // integers below 2^53 that is not whole lies at least 1/s from the next
  // whole number, more than its rounding error), held within +-(2^31 - 2^10)
  // so that window arithmetic stays in int32
  FSMI_DEV int block(double v) const {
    const double q = floor(floor(v) / (double)s);
    return (int)fmin(fmax(q, -2147482624.0), 2147482624.0);
  }
  // the pose's fraction inside its block along one axis, in [0, 1)
  FSMI_DEV float frac(double v) const {
    const double q = v / (double)s;
    return (float)(q - floor(q));
  }
  // block (bx, by) of the map, 0.5 outside (int32: the map has < 2^31 cells)
  FSMI_DEV float at(int bx, int by) const {
    const bool on = (unsigned)bx < (unsigned)X && (unsigned)by < (unsigned)Y;
    const float m = map[on ? bx + (int)X * by : 0];
    return on ? m : 0.5f;
  }
  // the resampled pixel from the four blocks around it (bx, by = the lower ones)
  FSMI_DEV float bilinear(int bx, int by, float fx, float fy) const {
    return lerp2(at(bx, by), at(bx + 1, by), at(bx, by + 1), at(bx + 1, by + 1), fx, fy);
  }
  // block and fraction of pose b, from the pose
  FSMI_DEV PatchOrigin origin_of_pose(int64_t b) const {
    const double x = poses[4 * b], y = poses[4 * b + 1];
    return PatchOrigin{block(x), block(y), frac(x), frac(y)};
  }
  // the same, from the batch's table (the patch kernels run after k_patch_origin)
  FSMI_DEV PatchOrigin origin(int64_t b) const { return org[b]; }
  // a, b: blocks (bx, by), (bx + 1, by); c, d: the row below
  static FSMI_DEV float lerp2(float a, float b, float c, float d, float fx, float fy) {
    const float top = fmaf(fx, b - a, a), bot = fmaf(fx, d - c, c);
    return fmaf(fy, bot - top, top);
  }
};

// Block means: out[v][u] = mean of the map's cells x in [s u, s u + s),
// y in [s v, s v + s) that lie inside the map (FP64 sum, fixed order).
__global__ void k_pool_map(const float* __restrict__ map, int64_t X, int64_t Y, int s,
                           int64_t Xc, int64_t Yc, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Xc * Yc;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = i % Xc, v = i / Xc;
    const int64_t x1 = min<int64_t>(s * u + s, X), y1 = min<int64_t>(s * v + s, Y);
    double acc = 0.0;
    for (int64_t y = s * v; y < y1; ++y)
      for (int64_t x = s * u; x < x1; ++x) acc += (double)map[x + X * y];
    out[i] = (float)(acc / (double)((x1 - s * u) * (y1 - s * v)));
  }
}

// PatchOrigin of each of the batch's n poses.
__global__ void k_patch_origin(int64_t n, PatchSrc src, PatchOrigin* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src.origin_of_pose(i);
}

// Two floats as packed BF16 (round to nearest even), low half first: one
// two-lane conversion instruction.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
FSMI_DEV uint32_t pack2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2{a, b}), bf16x2));
}

// ReLU of two floats, packed as BF16 (low half first): the two-lane
// conversion, then a two-lane 16-bit integer max with 0 on the bits.  A BF16
// value with its sign bit set, -0 included, is a negative int16 and becomes
// +0; rounding commutes with the max, so this is the packed ReLU of the
// floats.
typedef short shortx2 __attribute__((ext_vector_type(2)));
FSMI_DEV uint32_t pack2_relu(float a, float b) {
  const shortx2 v = __builtin_bit_cast(shortx2, __builtin_convertvector((floatx2{a, b}), bf16x2));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, (shortx2){0, 0}));
}

// ReLU signs of a stored activation for the next layer's input-gradient pass:
// word g of pixel p (sign[4 p + g]) holds, at bit 4 t + r, whether channel
// 16 t + 4 g + r is > 0, the channels lane group g holds in the forward and
// the input-gradient kernels alike (NT = channels / 16).
template <int NT> struct SignWord;
template <> struct SignWord<2> { typedef uint8_t type; };
template <> struct SignWord<4> { typedef uint16_t type; };
template <> struct SignWord<8> { typedef uint32_t type; };
// The 4 sign bits of two packed BF16 pairs (>= 0 values: > 0 iff not zero).
FSMI_DEV uint32_t sign4(uint2 w) {
  return ((w.x & 0xffffu) != 0u ? 1u : 0u) | ((w.x >> 16) != 0u ? 2u : 0u) |
         ((w.y & 0xffffu) != 0u ? 4u : 0u) | ((w.y >> 16) != 0u ? 8u : 0u);
}

// ---------------------------------------------------------------------------
// Forward convolutions after conv2 (k_conv3_rows, k_conv4_rows, k_conv5_rows)
// share these conventions.  Activations are BF16, pixel-major with the
// channels of a pixel contiguous (act[pixel][channel], pixels row-major per
// pose).  Products are taken transposed: the weights W[co][tap][ci] are the A
// operand (16 output channels x 32 input channels) and 16 output pixels' input
// channels the B operand, so D[n][p] leaves lane (i, g) with channels
// 16t + 4g .. + 3 of pixel i, stored as one 8-byte word, and the bias starts
// the accumulator.  In training the kernels also write the ReLU sign words of
// their output (SignWord layout above).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// conv3 (64 -> 64 channels, 32^2 -> 16^2) by input rows.  An output row is 16
// pixels, one per lane i of a lane group, so a wave takes four output rows oy0
// .. oy0 + 3 of one pose (a unit; four units per pose) and reads the nine
// input rows under them once each, in order: lane (i, g) loads the even
// column 2i and the odd column 2i + 1 of a row (channels 32c + 8g .. + 7, c =
// 0, 1), and the odd column left of 2i, 2i - 1, is the odd load of lane i - 1,
// one lane shift within the 16-lane row (lane 0 gets 0: the zero padding left
// of column 0).  Input row 2(oy0 + m) + ky is tap row ky of output row m, so a
// row feeds one or two output rows as it arrives, and no input byte is read
// twice by a wave (a tap-by-tap loop reads each 2.25 times, from all
// over the pose: 9 taps x 256 pixels x 128 bytes, and concurrent workgroups'
// poses exceed the L2, so most of it comes from HBM again).  All
// nine taps' weights sit in LDS as 72 fragments of 1 KiB (fragment (tap, c, t)
// = lane l's W[16t + l % 16][tap][32c + 8(l / 16) .. + 7] at 16 l), staged
// once by each persistent workgroup; the waves then run their units without
// barriers.
// ---------------------------------------------------------------------------
constexpr int kC3Waves = 4;                           // waves per workgroup
constexpr int kC3Frag = 512;                          // bf16 per weight fragment
constexpr int kC3WElems = 9 * 2 * 4 * kC3Frag;        // 72 KiB

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// lane i of each 16-lane row takes lane i - 1's value, lane 0 takes 0
FSMI_DEV bf16x8 shift_right1(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v), r;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    r[q] = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u[q], 0x111, 0xf, 0xf, false);   // row_shr:1
  return __builtin_bit_cast(bf16x8, r);
}

// The unit's 72 product groups in input-row order: group k is tap (ky, kx),
// channel half c, output row m (= (rr - ky) / 2) of input row rr, four
// products (one per 16-channel output tile).
struct Conv3Plan {
  int8_t rr[72], ky[72], kx[72], c[72];
  constexpr Conv3Plan() : rr(), ky(), kx(), c() {
    int k = 0;
    for (int r = 0; r < 9; ++r)
      for (int y = 0; y < 3; ++y) {
        if (r - y < 0 || ((r - y) & 1) || (r - y) / 2 >= 4) continue;
        for (int x = 0; x < 3; ++x)
          for (int h = 0; h < 2; ++h) {
            rr[k] = (int8_t)r;
            ky[k] = (int8_t)y;
            kx[k] = (int8_t)x;
            c[k] = (int8_t)h;
            ++k;
          }
      }
  }
};
constexpr Conv3Plan kC3Plan{};
constexpr int kC3Ahead = 3;   // input rows in flight beyond the one in use

__global__ __launch_bounds__(64 * kC3Waves, 2) void k_conv3_rows(int64_t n_units,
                                                                const bf16* __restrict__ in,
                                                                const bf16* __restrict__ W,
                                                                const float* __restrict__ bias,
                                                                bf16* __restrict__ out,
                                                                uint16_t* __restrict__ sign) {
  constexpr int HIN = 32, HOUT = 16, CIN = 64, COUT = 64, MT = 4, NR = 2 * MT + 1;
  __shared__ __align__(16) bf16 sW[kC3WElems];
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = lane & 15, g = lane >> 4;
  // fragment (tap, c, t), lane l: 16 bytes of W[co = 16t + l % 16][tap][32c + 8(l / 16) ..]
  for (int e = tid; e < kC3WElems / 8; e += 64 * kC3Waves) {
    const int l = e & 63, f = e >> 6, t = f & 3, c = (f >> 2) & 1, tap = f >> 3;
    *reinterpret_cast<bf16x8*>(sW + 8 * e) =
        load8(W + ((16 * t + (l & 15)) * 9 + tap) * CIN + 32 * c + 8 * (l >> 4));
  }
  __syncthreads();
  floatx4 bv[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) bv[t] = *reinterpret_cast<const floatx4*>(bias + 16 * t + 4 * g);
  // input row rr = 0 .. 8 of unit u is image row 2 oy0 - 1 + rr (<= 31; only
  // rr = 0 of a pose's top unit lies outside: zeros).  x[rr] = even column
  // c = 0, 1, then odd column c = 0, 1.  The last kC3Ahead rows' loads are
  // followed by the next unit's first rows, into the registers of the rows
  // already used, so no unit starts by waiting for memory.
  bf16x8 x[NR][4];
  auto fetch = [&](int64_t un, int rr, int slot) {
    const int row = 2 * (MT * (int)(un & 3)) - 1 + rr;
    const bool ok = row >= 0;
    const bf16* p = in + (((un >> 2) * HIN + (ok ? row : 0)) * HIN + 2 * i) * CIN + 8 * g;
#pragma unroll
    for (int q = 0; q < 4; ++q) x[slot][q] = load8(p + (q >> 1) * CIN + 32 * (q & 1));
    if (!ok) {
#pragma unroll
      for (int q = 0; q < 4; ++q) x[slot][q] = zero8();
    }
  };
  const int64_t wave0 = (int64_t)blockIdx.x * kC3Waves + __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * kC3Waves;
  if (wave0 < n_units) {
#pragma unroll
    for (int rr = 0; rr < kC3Ahead; ++rr) fetch(wave0, rr, rr);
  }
  for (int64_t u = wave0; u < n_units; u += n_waves) {
    const int64_t b = u >> 2, un = u + n_waves;
    const int oy0 = MT * (int)(u & 3);
    // the weight reads' base, opaque to the compiler: keeps it from hoisting
    // the 72 fragment reads out of the unit loop (288 registers)
    int wofs = 8 * lane;
    asm volatile("" : "+v"(wofs));
    floatx4 acc[MT][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m][t] = bv[t];
    bf16x8 ol[2];   // odd column left of 2i, of the row in use
    auto begin_row = [&](int k) {
      const int rr = kC3Plan.rr[k];
      if (k > 0 && kC3Plan.rr[k - 1] == rr) return;
      if (rr + kC3Ahead < NR) fetch(u, rr + kC3Ahead, rr + kC3Ahead);
      else if (un < n_units) fetch(un, rr + kC3Ahead - NR, rr + kC3Ahead - NR);
#pragma unroll
      for (int c = 0; c < 2; ++c) ol[c] = shift_right1(x[rr][2 + c]);
    };
    bf16x8 wa[4], wb[4];
    auto wload = [&](int k, bf16x8 (&w)[4]) {
      const int f = ((3 * kC3Plan.ky[k] + kC3Plan.kx[k]) * 2 + kC3Plan.c[k]) * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = *reinterpret_cast<const bf16x8*>(sW + (f + t) * kC3Frag + wofs);
    };
    auto products = [&](int k, const bf16x8 (&w)[4]) {
      const int rr = kC3Plan.rr[k], kx = kC3Plan.kx[k], c = kC3Plan.c[k];
      const int m = (rr - kC3Plan.ky[k]) >> 1;
      const bf16x8 xv = kx == 0 ? ol[c] : kx == 1 ? x[rr][c] : x[rr][2 + c];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[m][t] = mfma(w[t], xv, acc[m][t]);
    };
    wload(0, wa);
#pragma unroll
    for (int k = 0; k < 72; k += 2) {
      begin_row(k);
      wload(k + 1, wb);
      products(k, wa);
      __builtin_amdgcn_sched_barrier(0);
      begin_row(k + 1);
      if (k + 2 < 72) wload(k + 2, wa);
      products(k + 1, wb);
      __builtin_amdgcn_sched_barrier(0);
    }
    // D[n][p]: channels 16t + 4g + r of pixel (oy0 + m, i)
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int64_t pix = (b * HOUT + oy0 + m) * HOUT + i;
      bf16* op = out + pix * COUT + 4 * g;
      uint32_t bits = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint2 w;
        w.x = pack2_relu(acc[m][t][0], acc[m][t][1]);
        w.y = pack2_relu(acc[m][t][2], acc[m][t][3]);
        *reinterpret_cast<uint2*>(op + 16 * t) = w;
        bits |= sign4(w) << (4 * t);
      }
      if (sign) sign[4 * pix + g] = (uint16_t)bits;
    }
  }
}

// ---------------------------------------------------------------------------
// conv4 (64 -> 128 channels, 16^2 -> 8^2) in the same manner: a unit is
// output rows oy0, oy0 + 1 of one pose (four units per pose), lane (i, g) of
// a fragment pixel (oy0 + i / 8, i % 8), so tap row ky of the fragment reads
// input row 2 (oy0 + i / 8) + ky - 1 per lane, the even and odd columns
// 2 (i % 8) and 2 (i % 8) + 1, and the odd column to the left is a one-lane
// shift that leaves lanes i % 8 = 0 at 0 (the zero padding).  All nine
// taps' weights, 144 fragments of 1 KiB, fill one persistent workgroup's LDS
// (one workgroup of eight waves per compute unit); each wave loads its next
// unit's three tap rows while it computes the current one.
// ---------------------------------------------------------------------------
constexpr int kC4Waves = 8;
constexpr int kC4WElems = 9 * 2 * 8 * kC3Frag;       // 144 KiB

// lane i of each 16-lane row takes lane i - 1's value, ANDed with keep (all
// ones, or 0 for the first lane of a segment).  The lane shift must run with
// every lane active (a lane reads its neighbour's register, and an inactive
// neighbour gives 0), so the segment's first lane is cleared by the mask after
// it, never by a branch around it, which the compiler could form from a select.
FSMI_DEV bf16x8 shift_right1_masked(bf16x8 v, unsigned keep) {
  u32x4 u = __builtin_bit_cast(u32x4, shift_right1(v));
#pragma unroll
  for (int q = 0; q < 4; ++q) u[q] &= keep;
  return __builtin_bit_cast(bf16x8, u);
}

__global__ __launch_bounds__(64 * kC4Waves, 2) void k_conv4_rows(int64_t n_units,
                                                                const bf16* __restrict__ in,
                                                                const bf16* __restrict__ W,
                                                                const float* __restrict__ bias,
                                                                bf16* __restrict__ out,
                                                                uint32_t* __restrict__ sign) {
  constexpr int HIN = 16, HOUT = 8, CIN = 64, COUT = 128, NT = 8;
  __shared__ __align__(16) bf16 sW4[kC4WElems];
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = lane & 15, g = lane >> 4, h = i >> 3, ox = i & 7;
  const unsigned keep = 0u - (unsigned)(ox != 0);   // 0 for the first lane of an 8-lane segment
  // fragment (tap, c, t), lane l: 16 bytes of W[co = 16t + l % 16][tap][32c + 8(l / 16) ..]
  for (int e = tid; e < kC4WElems / 8; e += 64 * kC4Waves) {
    const int l = e & 63, f = e >> 6, t = f & 7, c = (f >> 3) & 1, tap = f >> 4;
    *reinterpret_cast<bf16x8*>(sW4 + 8 * e) =
        load8(W + ((16 * t + (l & 15)) * 9 + tap) * CIN + 32 * c + 8 * (l >> 4));
  }
  __syncthreads();
  floatx4 bv[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) bv[t] = *reinterpret_cast<const floatx4*>(bias + 16 * t + 4 * g);
  // x[ky] = even column c = 0, 1, then odd column c = 0, 1 of input row
  // 2 (oy0 + h) + ky - 1 (<= 15; < 0 only for h = 0, ky = 0 of a pose's top unit: zeros)
  bf16x8 x[3][4], nx[3][4];
  auto fetch = [&](int64_t un, bf16x8 (&d)[3][4]) {
    const int oy = 2 * (int)(un & 3) + h;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const int row = 2 * oy + ky - 1;
      const bool ok = row >= 0;
      const bf16* p = in + (((un >> 2) * HIN + (ok ? row : 0)) * HIN + 2 * ox) * CIN + 8 * g;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bf16x8 val = load8(p + (q >> 1) * CIN + 32 * (q & 1));
        d[ky][q] = ok ? val : zero8();
      }
    }
  };
  const int64_t wave0 = (int64_t)blockIdx.x * kC4Waves + __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * kC4Waves;
  if (wave0 < n_units) fetch(wave0, x);
  for (int64_t u = wave0; u < n_units; u += n_waves) {
    const int64_t un = u + n_waves;
    if (un < n_units) fetch(un, nx);
    int wofs = 8 * lane;   // opaque to the compiler: no hoisting of the fragment reads
    asm volatile("" : "+v"(wofs));
    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = bv[t];
    bf16x8 wa[NT], wb[NT];
    // group k = (ky, kx, c) in that order, 18 groups of NT products sharing one B operand
    auto wload = [&](int k, bf16x8 (&w)[NT]) {
      const int f = k * NT;   // (tap * 2 + c) * NT with tap = 3 ky + kx
#pragma unroll
      for (int t = 0; t < NT; ++t) w[t] = *reinterpret_cast<const bf16x8*>(sW4 + (f + t) * kC3Frag + wofs);
    };
    bf16x8 ol[3][2];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int c = 0; c < 2; ++c) ol[ky][c] = shift_right1_masked(x[ky][2 + c], keep);
    auto products = [&](int k, const bf16x8 (&w)[NT]) {
      const int c = k & 1, tap = k >> 1, ky = tap / 3, kx = tap % 3;
      const bf16x8 xv = kx == 0 ? ol[ky][c] : kx == 1 ? x[ky][c] : x[ky][2 + c];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma(w[t], xv, acc[t]);
    };
    wload(0, wa);
#pragma unroll
    for (int k = 0; k < 18; k += 2) {
      wload(k + 1, wb);
      products(k, wa);
      __builtin_amdgcn_sched_barrier(0);
      if (k + 2 < 18) wload(k + 2, wa);
      products(k + 1, wb);
      __builtin_amdgcn_sched_barrier(0);
    }
    // D[n][p]: channels 16t + 4g + r of pixel (oy0 + h, ox)
    const int64_t pix = ((u >> 2) * HOUT + 2 * (int)(u & 3) + h) * HOUT + ox;
    bf16* op = out + pix * COUT + 4 * g;
    uint32_t bits = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      uint2 w;
      w.x = pack2_relu(acc[t][0], acc[t][1]);
      w.y = pack2_relu(acc[t][2], acc[t][3]);
      *reinterpret_cast<uint2*>(op + 16 * t) = w;
      bits |= sign4(w) << (4 * t);
    }
    if (sign) sign[4 * pix + g] = bits;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int q = 0; q < 4; ++q) x[ky][q] = nx[ky][q];
  }
}

// ---------------------------------------------------------------------------
// conv5 (128 -> 128 channels, 8^2 -> 4^2) in the same manner.  A pose's 16
// output pixels are one fragment (lane i: pixel (i / 4, i % 4)), and the
// weights of all 128 output channels (288 KiB) exceed one workgroup's LDS, so
// a workgroup holds those of one half, output channels 64 chh .. 64 chh + 63
// (chh = its index % 2), and a unit is (pose, half).  Tap row ky of lane i
// reads input row 2 (i / 4) + ky - 1, columns 2 (i % 4) and 2 (i % 4) + 1,
// channels 32c + 8g .. + 7 (c = 0 .. 3); the odd column to the left is a
// lane shift that leaves lanes i % 4 = 0 at 0.  No sign words: the head's
// backward reads act5 itself.
// ---------------------------------------------------------------------------
constexpr int kC5Waves = 8;
constexpr int kC5WElems = 9 * 4 * 4 * kC3Frag;       // 144 KiB: one half's weights

__global__ __launch_bounds__(64 * kC5Waves, 2) void k_conv5_rows(int64_t n_poses,
                                                                const bf16* __restrict__ in,
                                                                const bf16* __restrict__ W,
                                                                const float* __restrict__ bias,
                                                                bf16* __restrict__ out) {
  constexpr int HIN = 8, CIN = 128, COUT = 128, KC = 4, NT = 4;
  __shared__ __align__(16) bf16 sW5[kC5WElems];
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = lane & 15, g = lane >> 4, oy = i >> 2, ox = i & 3;
  const unsigned keep = 0u - (unsigned)(ox != 0);   // 0 for the first lane of a 4-lane segment
  const int chh = (int)(blockIdx.x & 1);
  // fragment (tap, c, t), lane l: 16 bytes of W[co = 64 chh + 16t + l % 16][tap][32c + 8(l / 16) ..]
  for (int e = tid; e < kC5WElems / 8; e += 64 * kC5Waves) {
    const int l = e & 63, f = e >> 6, t = f & 3, c = (f >> 2) & 3, tap = f >> 4;
    *reinterpret_cast<bf16x8*>(sW5 + 8 * e) =
        load8(W + ((64 * chh + 16 * t + (l & 15)) * 9 + tap) * CIN + 32 * c + 8 * (l >> 4));
  }
  __syncthreads();
  floatx4 bv[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) bv[t] = *reinterpret_cast<const floatx4*>(bias + 64 * chh + 16 * t + 4 * g);
  // x[ky] = even column c = 0 .. 3, then odd column c = 0 .. 3 of input row
  // 2 oy + ky - 1 (<= 7; < 0 only for oy = 0, ky = 0: zeros)
  bf16x8 x[3][2 * KC];
  auto fetch = [&](int64_t b) {
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const int row = 2 * oy + ky - 1;
      const bool ok = row >= 0;
      const bf16* p = in + ((b * HIN + (ok ? row : 0)) * HIN + 2 * ox) * CIN + 8 * g;
#pragma unroll
      for (int q = 0; q < 2 * KC; ++q) {
        const bf16x8 val = load8(p + (q / KC) * CIN + 32 * (q % KC));
        x[ky][q] = ok ? val : zero8();
      }
    }
  };
  // workgroups 2w and 2w + 1 take the two halves of the same poses
  const int64_t wave0 = (int64_t)(blockIdx.x >> 1) * kC5Waves + __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n_waves = (int64_t)(gridDim.x >> 1) * kC5Waves;
  for (int64_t b = wave0; b < n_poses; b += n_waves) {
    fetch(b);
    int wofs = 8 * lane;   // opaque to the compiler: no hoisting of the fragment reads
    asm volatile("" : "+v"(wofs));
    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = bv[t];
    bf16x8 wa[NT], wb[NT];
    // group k = (tap, c), 36 groups of NT products sharing one B operand
    auto wload = [&](int k, bf16x8 (&w)[NT]) {
#pragma unroll
      for (int t = 0; t < NT; ++t) w[t] = *reinterpret_cast<const bf16x8*>(sW5 + (k * NT + t) * kC3Frag + wofs);
    };
    auto products = [&](int k, const bf16x8 (&w)[NT]) {
      const int c = k % KC, tap = k / KC, ky = tap / 3, kx = tap % 3;
      const bf16x8 xo = x[ky][KC + c];
      const bf16x8 xv = kx == 1 ? x[ky][c] : kx == 2 ? xo : shift_right1_masked(xo, keep);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma(w[t], xv, acc[t]);
    };
    wload(0, wa);
#pragma unroll
    for (int k = 0; k < 9 * KC; k += 2) {
      wload(k + 1, wb);
      products(k, wa);
      __builtin_amdgcn_sched_barrier(0);
      if (k + 2 < 9 * KC) wload(k + 2, wa);
      products(k + 1, wb);
      __builtin_amdgcn_sched_barrier(0);
    }
    // D[n][p]: channels 64 chh + 16t + 4g + r of pixel (oy, ox)
    const int64_t pix = (b * 4 + oy) * 4 + ox;
    bf16* op = out + pix * COUT + 64 * chh + 4 * g;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      uint2 w;
      w.x = pack2_relu(acc[t][0], acc[t][1]);
      w.y = pack2_relu(acc[t][2], acc[t][3]);
      *reinterpret_cast<uint2*>(op + 16 * t) = w;
    }
  }
}

// ---------------------------------------------------------------------------
// conv1 fused into conv2 (inference and training).  A workgroup owns 8 x 8 output pixels of
// conv2 (all 64 channels) at a time: it gathers the 35 x 35 patch window those
// pixels depend on, computes the 17 x 17 x 32 conv1 outputs of the window into
// LDS (zero where conv1's 64 x 64 grid ends: conv2's zero padding), then conv2
// from LDS, so conv1's activations never reach HBM.  The products are taken
// transposed (weights as the A operand, activations as B), so a lane ends with
// four consecutive channels of one pixel and stores them as one 8-byte word.
// Persistent workgroups keep W1 in registers, and each wave the W2 fragments
// of its 32 output channels; the tiles run as a two-stage pipeline over
// double-buffered LDS (described at the loop).  In training (SAVE) the kernel
// also stores conv1's activations and both layers' ReLU sign words for the
// backward pass: a tile owns the conv1 pixels of window rows and columns
// 1 .. 16 (conv1 rows 2 oy0 .. 2 oy0 + 15; row 0 of the window belongs to the
// tile above), so each conv1 pixel is stored once.  conv1's nine taps take one
// v_mfma_f32_16x16x16_bf16 per channel tile (K = 16, the slot layout given
// where W1 is loaded).
// ---------------------------------------------------------------------------
constexpr int kT2 = 8;                 // conv2 tile edge (output pixels)
constexpr int kT1 = 2 * kT2 + 1;       // 17: conv1 window edge
constexpr int kTP = 2 * kT1 + 1;       // 35: patch window edge
constexpr int kA1Px = 40;              // bf16 per conv1 pixel in LDS (32 channels + 8 pad)
constexpr int kC1Tiles = 20;           // conv1 column tiles of 16 pixels per window (19 needed)
constexpr int kPWin = kTP * kTP + 11;   // patch window in LDS: 1225 pixels, zero padding, 8-byte rows
constexpr int kPatchPer = (kTP * kTP + 255) / 256;   // gathers per thread

// A thread's share of a tile's patch window: element e = tid + 256 k at row
// e / kTP, column e % kTP, the same for every tile (computed once).
struct WinOffs {
  int r[kPatchPer], c[kPatchPer];
  bool v[kPatchPer];
};
FSMI_DEV WinOffs win_offsets(int tid) {
  WinOffs w;
#pragma unroll
  for (int k = 0; k < kPatchPer; ++k) {
    const int e = tid + 256 * k;
    w.v[k] = e < kTP * kTP;
    w.r[k] = w.v[k] ? e / kTP : 0;
    w.c[k] = w.v[k] ? e - (e / kTP) * kTP : 0;
  }
  return w;
}

// Patch window of tile `tile` into registers: all gathers issue before any is
// used (clamped addresses, selects after the loads).  The map has fewer than
// 2^31 cells, so cell arithmetic is int32.
FSMI_DEV void gather_window(const PatchSrc& src, int64_t tile, const WinOffs& w,
                            float (&v)[kPatchPer]) {
  const int64_t b = tile >> 4;
  const int oy0 = kT2 * (int)((tile >> 2) & 3), ox0 = kT2 * (int)(tile & 3);
  const int py0 = 4 * oy0 - 3, px0 = 4 * ox0 - 3;   // patch window origin
  const PatchOrigin og = src.origin(b);
  const int cx0 = og.bx - kPatch / 2 + px0;
  const int cy0 = og.by - kPatch / 2 + py0;
  const float fx = og.fx, fy = og.fy;
  // window rows and columns before the patch's first (the window never
  // reaches past its last: py0, px0 <= 93 and 93 + 34 < 128)
  const int rmin = py0 < 0 ? -py0 : 0, cmin = px0 < 0 ? -px0 : 0;
  if (cx0 >= 0 && cy0 >= 0 && cx0 + kTP < src.X && cy0 + kTP < src.Y) {
    // every block the window reads lies inside the map: no per-block checks
    const float* base = src.map + (cx0 + src.X * (int64_t)cy0);
    const uint32_t X = (uint32_t)src.X;
#pragma unroll
    for (int k = 0; k < kPatchPer; ++k) {
      const uint32_t o = (uint32_t)w.r[k] * X + (uint32_t)w.c[k];
      const float m = PatchSrc::lerp2(base[o], base[o + 1], base[o + X], base[o + X + 1], fx, fy);
      v[k] = w.r[k] >= rmin && w.c[k] >= cmin ? m : 0.0f;
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < kPatchPer; ++k) {
    const float m = src.bilinear(cx0 + w.c[k], cy0 + w.r[k], fx, fy);
    v[k] = w.r[k] >= rmin && w.c[k] >= cmin ? m : 0.0f;
  }
}

template <bool SAVE>
__global__ __launch_bounds__(256) void k_conv12_fwd(int64_t n_tiles, PatchSrc src,
                                                    const bf16* __restrict__ W1,
                                                    const float* __restrict__ b1,
                                                    const bf16* __restrict__ W2,
                                                    const float* __restrict__ b2,
                                                    bf16* __restrict__ act2,
                                                    bf16* __restrict__ act1,
                                                    uint8_t* __restrict__ sign1,
                                                    uint16_t* __restrict__ sign2) {
  __shared__ __align__(16) bf16 sP[2][kPWin];
  // conv1 buffers hold 20 column tiles of 16 pixels: the window's 289 and
  // padding that the waves' fifth column tiles write without a branch
  __shared__ __align__(16) bf16 sA1[2][kC1Tiles * 16 * kA1Px];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 15, g = lane >> 4;
  // conv2: wave w takes column tiles 2 ph, 2 ph + 1 of the tile's 64 pixels and
  // output channel tiles 2 chh, 2 chh + 1 (ph = w % 2, chh = w / 2).  Its A
  // operands, W2[16 (2 chh + tt) + i][tap][8g .. 8g + 7], stay in registers for
  // the whole launch (W2 is [co][tap][ci], 32 input channels).
  const int ph = wave & 1, chh = wave >> 1;
  bf16x8 w2r[9][2];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) w2r[tap][tt] = load8(W2 + ((16 * (2 * chh + tt) + i) * 9 + tap) * 32 + 8 * g);
  // conv1 as a 16 x 16 x 16 product: A[n][k] = W1[16t + n][tap(k)], B[k][p] =
  // the window pixel under tap(k) of conv1 pixel p.  The K slots are laid out
  // so that lane group g reads its four B values as two aligned pairs of
  // window pixels (two 4-byte LDS reads at offsets off0, off1 from the
  // pixel's base, which is even): g = 0 takes taps (0,0) (0,1) | (0,2) -,
  // g = 1 (1,1) (1,2) | - (1,0), g = 2 (2,0) (2,1) | (2,2) -, g = 3 nothing.
  // A "-" slot has weight 0 and reads a neighbouring window pixel or the
  // zeroed padding after the window: finite values, so the sum is the one
  // over the nine taps.
  bf16x4 w1[2];
  int slot_tap[4];   // tap (3 ky + kx) of slot 4g + q, -1 for none
  {
    constexpr int kSlotTap[4][4] = {{0, 1, 2, -1}, {4, 5, -1, 3}, {6, 7, 8, -1}, {-1, -1, -1, -1}};
#pragma unroll
    for (int q = 0; q < 4; ++q) slot_tap[q] = kSlotTap[g][q];
  }
  const int off0 = g == 1 ? kTP + 1 : g == 2 ? 2 * kTP : 0;
  const int off1 = g == 0 ? 2 : g == 1 ? kTP - 1 : g == 2 ? 2 * kTP + 2 : 0;
  float bias1[2][4], bias2[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w1[t][q] = slot_tap[q] >= 0 ? W1[(16 * t + i) * 9 + slot_tap[q]] : (bf16)0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias1[t][r] = b1[16 * t + 4 * g + r];
  }
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) bias2[tt][r] = b2[16 * (2 * chh + tt) + 4 * g + r];
  const WinOffs woff = win_offsets(tid);
  // conv1 pixels of this lane (p = 16 m + i, m = wave, wave + 4, ...): their
  // place in the window and their patch offset, the same for every tile.
  // Every wave takes five column tiles; pixels past the window's 289 (the
  // last tile and a half) read the patch at 0 and write padding slots.
  constexpr int kUPerWave = kC1Tiles / 4;   // conv1 column tiles per wave
  int c1_pr[kUPerWave], c1_pc[kUPerWave], c1_base[kUPerWave];
#pragma unroll
  for (int u = 0; u < kUPerWave; ++u) {
    const int p = 16 * (wave + 4 * u) + i;
    const bool pv = p < kT1 * kT1;
    c1_pr[u] = pv ? p / kT1 : -1000;          // -1000: outside any grid
    c1_pc[u] = pv ? p - (p / kT1) * kT1 : 0;
    c1_base[u] = pv ? 2 * c1_pr[u] * kTP + 2 * c1_pc[u] : 0;
  }
  // Two-stage pipeline over the workgroup's tiles j = 0, 1, ...: step j runs
  // conv1 of tile j (patch buffer j % 2 -> conv1 buffer j % 2) beside conv2
  // of tile j - 1 (conv1 buffer (j - 1) % 2), stores tile j + 1's patch
  // window, gathered during step j - 1, into patch buffer (j + 1) % 2 and
  // issues the gathers of tile j + 2; one barrier ends the step.  Each buffer
  // is written in one step and read in the next only.  A workgroup's tiles
  // are one contiguous run, so a pose's 16 tiles follow each other and their
  // overlapping windows meet the same map blocks in the caches.
  const int64_t per = (n_tiles + gridDim.x - 1) / gridDim.x;
  const int64_t first = (int64_t)blockIdx.x * per;
  const int64_t n_my = first < n_tiles ? min<int64_t>(per, n_tiles - first) : 0;
  auto tile_of = [&](int64_t j) { return first + j; };
  float v[kPatchPer];
  auto stage_patch = [&](int buf) {
#pragma unroll
    for (int k = 0; k < kPatchPer; ++k) {
      const int e = tid + 256 * k;
      if (e < kTP * kTP) sP[buf][e] = (bf16)v[k];
    }
  };
  if (tid < 2 * (kPWin - kTP * kTP)) sP[tid & 1][kTP * kTP + (tid >> 1)] = (bf16)0.0f;   // padding
  if (n_my > 0) {
    gather_window(src, tile_of(0), woff, v);
    stage_patch(0);
    if (n_my > 1) gather_window(src, tile_of(1), woff, v);
  }
  __syncthreads();
  // conv1 on the window of tile j: 289 pixels in 20 column tiles of 16, five per wave
  auto conv1_tile = [&](int64_t j) {
    const int64_t tile = tile_of(j);
    const int64_t b = tile >> 4;
    const int oy0 = kT2 * (int)((tile >> 2) & 3), ox0 = kT2 * (int)(tile & 3);
    const bf16* P = sP[j & 1];
    bf16* A1 = sA1[j & 1];
    // B operands of all five column tiles first (the window pixels of slots
    // 4g .. 4g + 3 of each pixel): the compiler cannot tell the patch buffer
    // from the conv1 buffer written below, so reads placed after a write
    // would wait for it
    bf16x4 xs[kUPerWave];
#pragma unroll
    for (int u = 0; u < kUPerWave; ++u) {
      uint2 xw;
      xw.x = *reinterpret_cast<const uint32_t*>(P + c1_base[u] + off0);
      xw.y = *reinterpret_cast<const uint32_t*>(P + c1_base[u] + off1);
      xs[u] = __builtin_bit_cast(bf16x4, xw);
    }
#pragma unroll
    for (int u = 0; u < kUPerWave; ++u) {
      const int p = 16 * (wave + 4 * u) + i;
      const bool pv = c1_pr[u] >= 0;
      const int pr = pv ? c1_pr[u] : 0, pc = c1_pc[u];
      const bf16x4 x = xs[u];
      const int y1 = 2 * oy0 - 1 + pr, x1 = 2 * ox0 - 1 + pc;
      const bool inside = pv && y1 >= 0 && y1 < 64 && x1 >= 0 && x1 < 64;
      const bool owned = SAVE && pv && pr >= 1 && pc >= 1;   // implies inside
      const int64_t pix1 = (b * 64 + y1) * 64 + x1;
      uint32_t bits = 0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // D[n][p]: channels 16t + 4g + r of pixel p, the bias as the accumulator's start
        const floatx4 d = mfma16(w1[t], x, floatx4{bias1[t][0], bias1[t][1], bias1[t][2], bias1[t][3]});
        uint2 w;
        w.x = inside ? pack2_relu(d[0], d[1]) : 0u;
        w.y = inside ? pack2_relu(d[2], d[3]) : 0u;
        *reinterpret_cast<uint2*>(A1 + p * kA1Px + 16 * t + 4 * g) = w;
        if (owned) {
          *reinterpret_cast<uint2*>(act1 + pix1 * 32 + 16 * t + 4 * g) = w;
          bits |= sign4(w) << (4 * t);
        }
      }
      if (owned) sign1[4 * pix1 + g] = (uint8_t)bits;
    }
  };
  // conv2 of tile j: pixels 16 (2 ph + mm) + i of the 8 x 8 tile, channel tiles 2 chh + tt
  auto conv2_tile = [&](int64_t j) {
    const int64_t tile = tile_of(j);
    const int64_t b = tile >> 4;
    const int oy0 = kT2 * (int)((tile >> 2) & 3), ox0 = kT2 * (int)(tile & 3);
    const bf16* A1 = sA1[j & 1];
    floatx4 acc[2][2];   // the bias as the accumulators' start
    int qy[2], qx[2];
#pragma unroll
    for (int mm = 0; mm < 2; ++mm) {
      const int p = 16 * (2 * ph + mm) + i;
      qy[mm] = p >> 3;
      qx[mm] = p & 7;
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
        acc[mm][tt] = floatx4{bias2[tt][0], bias2[tt][1], bias2[tt][2], bias2[tt][3]};
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap % 3;
#pragma unroll
      for (int mm = 0; mm < 2; ++mm) {
        const bf16x8 x = load8(A1 + ((2 * qy[mm] + ky) * kT1 + 2 * qx[mm] + kx) * kA1Px + 8 * g);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) acc[mm][tt] = mfma(w2r[tap][tt], x, acc[mm][tt]);
      }
    }
#pragma unroll
    for (int mm = 0; mm < 2; ++mm) {
      const int64_t pix2 = (b * 32 + oy0 + qy[mm]) * 32 + ox0 + qx[mm];
      bf16* op = act2 + pix2 * 64 + 4 * g;
      uint32_t bits = 0;
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        uint2 w;
        w.x = pack2_relu(acc[mm][tt][0], acc[mm][tt][1]);
        w.y = pack2_relu(acc[mm][tt][2], acc[mm][tt][3]);
        *reinterpret_cast<uint2*>(op + 16 * (2 * chh + tt)) = w;
        bits |= sign4(w) << (4 * tt);
      }
      // byte chh of the pixel's 16-bit sign word g: channel tiles 2 chh, 2 chh + 1
      if (SAVE) reinterpret_cast<uint8_t*>(sign2)[2 * (4 * pix2 + g) + chh] = (uint8_t)bits;
    }
  };
  // The steps between the first and the last hold both stages in one basic
  // block, so the compiler interleaves conv1's VALU work with conv2's
  // products; their gathers are clamped to the last tile (a step past it
  // gathers and stages a window that nothing reads).
  if (n_my > 0) {
    conv1_tile(0);
    if (n_my > 1) {
      stage_patch(1);
      gather_window(src, tile_of(min<int64_t>(2, n_my - 1)), woff, v);
    }
  }
  __syncthreads();
  for (int64_t j = 1; j < n_my; ++j) {
    conv2_tile(j - 1);   // its LDS reads ahead of conv1's writes (another buffer)
    conv1_tile(j);
    stage_patch((j + 1) & 1);
    gather_window(src, tile_of(min<int64_t>(j + 2, n_my - 1)), woff, v);
    __syncthreads();
  }
  if (n_my > 0) conv2_tile(n_my - 1);
}

// ---------------------------------------------------------------------------
// Input-gradient pass: d_in[p][ci] = [act_in[p][ci] > 0] *
//   sum over taps and co of W[co][tap][ci] d_out[o][co], over the taps whose
//   output pixel o = ((iy + 1 - ky) / 2, (ix + 1 - kx) / 2) is whole and inside
//   the output grid.  With stride 2 and padding 1 those taps depend only on
//   the parity of the input pixel: an even row takes ky = 1 (oy = iy / 2), an
//   odd row ky = 0 (oy = (iy + 1) / 2) and ky = 2 (oy = (iy - 1) / 2); columns
//   alike.  So the input pixels fall into four classes of 1, 2, 2 and 4 taps,
//   and a wave takes pixels of one class only: no product is spent on a tap
//   that does not reach its pixels.  A workgroup is the four classes (one wave
//   each) of 16 MT consecutive half-resolution positions q = (b, a, c), pixel
//   (iy, ix) = (2 a + py, 2 c + px).  Products are taken transposed (weights
//   as the A operand, Wt is [tap][ci][co]), so a lane ends with four
//   consecutive channels of one pixel and loads and stores 8 bytes at once.
//   The d_out pixels a tile reads, (b, a + dy, c + dx) with dy, dx in {0, 1},
//   are the tile's own positions and the row after them: a contiguous range
//   of d_out, staged once in LDS for the four waves (each reads it about 2.25
//   times over).  nq = batch x (HIN / 2)^2 is a multiple of 16, and tiles
//   start on row boundaries.
// With WG1 (conv2's pass, whose d_in is d_out of conv1) the pass also takes
//   conv1's weight gradient, so conv1's d_out never reaches HBM: a workgroup
//   runs tiles_per_wg consecutive tiles, and each tile writes its 256 masked
//   BF16 gradients (the values d_in would hold) channel-major into LDS, stages
//   the 9 patch rows under its 4 conv1 rows, and adds to partial[s][co][col] =
//   sum over the tile's pixels p of d_in[p][co] B[p][col], col = tap (the
//   patch pixel under the tap), 9 (1: the bias) or 10..15 (0), the layout of
//   the later layers' weight-gradient partials, s = the workgroup.  Its four
//   waves take alternate 32-pixel steps; their sums are added in wave order at
//   the end, so the result is deterministic.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int HIN>
constexpr int dgrad_mt() { return CIN >= 128 ? 2 : 4; }
// WG1 workgroups per compute unit: the kernel is held to 4 waves per SIMD, so
// 4 workgroups of 4 waves fill a compute unit, and one such round of
// workgroups is the grid (each takes an equal run of tiles)
constexpr int kWg1PerCu = 4;

template <int CIN, int COUT, int HIN, bool WG1>
__global__ __launch_bounds__(256, WG1 ? 4 : 1) void k_conv_dgrad(int64_t nq, int tiles_per_wg,
                                                    const bf16* __restrict__ dout,
                                                    const bf16* __restrict__ Wt,
                                                    const bf16* __restrict__ act_in,
                                                    const void* __restrict__ sign,
                                                    bf16* __restrict__ din, PatchSrc src,
                                                    float* __restrict__ part) {
  constexpr int HOUT = HIN / 2, NT = CIN / 16, KC = COUT / 32, MT = dgrad_mt<CIN, COUT, HIN>();
  constexpr int TQ = 16 * MT, ROWD = COUT + 8;   // positions per tile; LDS row (one d_out pixel)
  static_assert(TQ % HOUT == 0, "tiles hold whole rows");
  static_assert(!WG1 || (CIN == 32 && HIN == 64 && TQ == 2 * HOUT && HIN * 2 == kPatch),
                "WG1: conv2's pass, tiles of two half-resolution rows (4 conv1 rows)");
  // WG1: KW = 4 TQ pixels per tile (the K of conv1's weight-gradient products),
  // stored channel-major with rows of KW + 8; SROW: a patch row with a zero
  // column on each side
  constexpr int KW = 4 * TQ, ROWA = KW + 8, SROW = kPatch + 2;
  __shared__ __align__(16) bf16 sD[(TQ + HOUT) * ROWD];
  __shared__ __align__(16) bf16 sA[WG1 ? CIN * ROWA : 8];
  __shared__ __align__(16) bf16 sPt[WG1 ? 9 * SROW : 8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int cls = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int py = cls >> 1, px = cls & 1;
  const int i = lane & 15, g = lane >> 4;
  const int64_t n_tiles = (nq + TQ - 1) / TQ;
  const int64_t tile0 = (int64_t)blockIdx.x * tiles_per_wg;
  // without WG1 a workgroup takes one tile (tiles_per_wg is 1 and the grid is n_tiles)
  const int64_t tile1 = WG1 ? min<int64_t>(tile0 + tiles_per_wg, n_tiles) : tile0 + 1;
  floatx4 accw[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) accw[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int64_t tile = tile0; tile < tile1; ++tile) {
    const int64_t base = tile * TQ;
    const int n_mt = (int)min<int64_t>(MT, (nq - base) / 16);   // >= 1: nq is a multiple of 16
    int64_t qb[MT];
    int qa[MT], qc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int64_t q = min<int64_t>(base + 16 * m + i, nq - 1);
      qb[m] = q / (HOUT * HOUT);
      qa[m] = (int)((q / HOUT) % HOUT);
      qc[m] = (int)(q % HOUT);
    }
    // the ReLU sign words (SignWord) of this lane's pixels, issued first so
    // that their latency overlaps the staging and the products
    typedef typename SignWord<NT>::type S;
    uint32_t sbm[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int64_t p = (qb[m] * HIN + 2 * qa[m] + py) * HIN + 2 * qc[m] + px;
      sbm[m] = sign ? (uint32_t)reinterpret_cast<const S*>(sign)[4 * p + g] : 0u;
    }
    __syncthreads();   // the previous tile's LDS reads are done
    for (int e = tid; e < (TQ + HOUT) * (COUT / 8); e += 256) {
      const int px8 = e / (COUT / 8), c8 = e % (COUT / 8);
      const int64_t q = base + px8;
      *reinterpret_cast<bf16x8*>(sD + px8 * ROWD + 8 * c8) = q < nq ? load8(dout + q * COUT + 8 * c8) : zero8();
    }
    if constexpr (WG1) {
      // staged row r = patch row 4 a0 - 1 + r (a0: the tile's first half-row),
      // staged column c = patch column c - 1, read from the map (PatchSrc)
      const int64_t b0 = base / (HOUT * HOUT);
      const int a0 = (int)((base / HOUT) % HOUT);
      const PatchOrigin og = src.origin(b0);
      const int mx0 = og.bx - kPatch / 2;
      const int my0 = og.by - kPatch / 2;
      const float fx = og.fx, fy = og.fy;
      // blocks mx0 - 1 .. mx0 + kPatch + 1 and my0 + 4 a0 - 1 .. my0 + 4 a0 + 8
      // inside the map: no per-block checks
      const int ry0 = my0 + 4 * a0 - 1;
      if (mx0 >= 1 && ry0 >= 0 && mx0 + kPatch + 1 < src.X && ry0 + 9 < src.Y) {
        const float* mp = src.map + ((mx0 - 1) + src.X * (int64_t)ry0);   // staged (0, 0)
        const uint32_t X = (uint32_t)src.X;
        for (int e = tid; e < 9 * SROW; e += 256) {
          const int r = e / SROW, c = e - r * SROW;
          const int iy = 4 * a0 - 1 + r, ix = c - 1;
          const uint32_t o = (uint32_t)r * X + (uint32_t)c;
          const float m = PatchSrc::lerp2(mp[o], mp[o + 1], mp[o + X], mp[o + X + 1], fx, fy);
          sPt[e] = (bf16)((unsigned)iy < (unsigned)kPatch && (unsigned)ix < (unsigned)kPatch ? m : 0.0f);
        }
      } else {
        for (int e = tid; e < 9 * SROW; e += 256) {
          const int r = e / SROW, c = e - r * SROW;
          const int iy = 4 * a0 - 1 + r, ix = c - 1;
          float v = 0.0f;
          if ((unsigned)iy < (unsigned)kPatch && (unsigned)ix < (unsigned)kPatch)
            v = src.bilinear(mx0 + ix, my0 + iy, fx, fy);
          sPt[e] = (bf16)v;
        }
      }
    }
    __syncthreads();
    floatx4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int nky = 1 + py, nkx = 1 + px;
#pragma unroll 1
    for (int jy = 0; jy < nky; ++jy) {
#pragma unroll 1
      for (int jx = 0; jx < nkx; ++jx) {
        // odd row: ky = 0 reads output row a + 1, ky = 2 row a; even row: ky = 1, row a
        const int ky = py ? 2 * jy : 1, kx = px ? 2 * jx : 1;
        const int dy = (py && jy == 0) ? 1 : 0, dx = (px && jx == 0) ? 1 : 0;
        const int tap = 3 * ky + kx;
        bf16x8 a[MT][KC];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          // d_out pixel (b, a + dy, c + dx) = position q + dy HOUT + dx
          const bool ok = m < n_mt && qa[m] + dy < HOUT && qc[m] + dx < HOUT;
          const bf16* dp = sD + (ok ? 16 * m + i + dy * HOUT + dx : 0) * ROWD;
#pragma unroll
          for (int c = 0; c < KC; ++c)
            a[m][c] = ok ? *reinterpret_cast<const bf16x8*>(dp + 32 * c + 8 * g) : zero8();
        }
#pragma unroll
        for (int c = 0; c < KC; ++c)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const bf16x8 w = load8(Wt + (tap * CIN + 16 * t + i) * COUT + 32 * c + 8 * g);
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m][t] = mfma(w, a[m][c], acc[m][t]);
          }
      }
    }
    // D[4 g + r][i]: channel 16 t + 4 g + r of pixel (m, i)
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if (m >= n_mt) {
        if constexpr (WG1) {   // positions past nq add nothing
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) sA[(16 * t + 4 * g + r) * ROWA + cls * TQ + 16 * m + i] = (bf16)0.0f;
          continue;
        } else {
          break;
        }
      }
      const int iy = 2 * qa[m] + py, ix = 2 * qc[m] + px;
      const int64_t p = (qb[m] * HIN + iy) * HIN + ix;
      // with sign words: bit 4 t + r of word g
      const uint32_t sb = sbm[m];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int ci = 16 * t + 4 * g;
        float mk[4];
        if (sign) {
#pragma unroll
          for (int r = 0; r < 4; ++r) mk[r] = (sb >> (4 * t + r)) & 1u ? 1.0f : 0.0f;
        } else {
          const uint2 av = *reinterpret_cast<const uint2*>(act_in + p * CIN + ci);
          // the BF16 activations widened to FP32 (the low half first)
          const uint32_t aw[2] = {av.x, av.y};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            mk[2 * h] = __builtin_bit_cast(float, aw[h] << 16) > 0.0f ? 1.0f : 0.0f;
            mk[2 * h + 1] = __builtin_bit_cast(float, aw[h] & 0xffff0000u) > 0.0f ? 1.0f : 0.0f;
          }
        }
        const uint2 w = uint2{pack2(acc[m][t][0] * mk[0], acc[m][t][1] * mk[1]),
                              pack2(acc[m][t][2] * mk[2], acc[m][t][3] * mk[3])};
        if constexpr (WG1) {
          // channel-major: row = channel, column = class, then position in the tile
          uint16_t* sa = reinterpret_cast<uint16_t*>(sA) + ci * ROWA + cls * TQ + 16 * m + i;
          sa[0] = (uint16_t)(w.x & 0xffffu);
          sa[ROWA] = (uint16_t)(w.x >> 16);
          sa[2 * ROWA] = (uint16_t)(w.y & 0xffffu);
          sa[3 * ROWA] = (uint16_t)(w.y >> 16);
        } else {
          *reinterpret_cast<uint2*>(din + p * CIN + ci) = w;
        }
      }
    }
    if constexpr (WG1) {
      __syncthreads();   // sA holds the tile's 256 pixels
      bf16x8 ones;
#pragma unroll
      for (int q = 0; q < 8; ++q) ones[q] = (bf16)1.0f;
      const int ky = i / 3, kx = i - 3 * (i / 3);
#pragma unroll
      for (int u = 0; u < KW / 128; ++u) {
        // pixels k = 32 ks + 8 g + j (j < 8): class kc, positions kq0 + j of the
        // tile, i.e. half-row a0 + da, columns c0 + j of that class
        const int ks = cls + 4 * u;
        const int k0 = 32 * ks + 8 * g, kc = k0 / TQ, kq0 = k0 - kc * TQ;
        const int da = kq0 / HOUT, c0 = kq0 - da * HOUT;
        bf16x8 fb;
        if (i < 9) {
          const bf16* sp = sPt + (4 * da + 2 * (kc >> 1) + ky) * SROW + 4 * c0 + 2 * (kc & 1) + kx;
#pragma unroll
          for (int j = 0; j < 8; ++j) fb[j] = sp[4 * j];
        } else {
          fb = i == 9 ? ones : zero8();
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bf16x8 fa = *reinterpret_cast<const bf16x8*>(sA + (16 * t + i) * ROWA + 32 * ks + 8 * g);
          accw[t] = mfma(fa, fb, accw[t]);
        }
      }
    }
  }   // tiles
  if constexpr (WG1) {
    __syncthreads();   // every wave is done with sA
    floatx4* red = reinterpret_cast<floatx4*>(sA);   // [wave][t][lane]
    static_assert(4 * NT * 64 * sizeof(floatx4) <= sizeof(bf16) * CIN * ROWA, "red fits in sA");
#pragma unroll
    for (int t = 0; t < NT; ++t) red[(cls * NT + t) * 64 + lane] = accw[t];
    __syncthreads();
    if (cls == 0) {
      // D[4 g + r][i]: co = 16 t + 4 g + r, column i
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const floatx4 d = ((red[t * 64 + lane] + red[(NT + t) * 64 + lane]) + red[(2 * NT + t) * 64 + lane]) +
                          red[(3 * NT + t) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[((int64_t)blockIdx.x * CIN + 16 * t + 4 * g + r) * 16 + i] = d[r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight-gradient pass, layers after the first: partial[s][co][tap CIN + ci] =
//   sum over the output pixels p of split s of d_out[p][co] x[p, tap][ci],
//   x[p, tap] the input pixel under tap `tap` of p (0 in the padding), and
//   partial[s][co][9 CIN] = sum_p d_out[p][co] (the bias).
// The sum runs over pixels, the K axis of the products, while both operands
// are stored channel-fastest.  So a workgroup stages 32 pixels at a time in
// LDS channel-major (the 32 pixels of a channel contiguous): a thread loads 4
// pixels x 8 channels (four 16-byte loads), transposes them in registers and
// writes 8 rows of 4 pixels; fragments are then single 16-byte LDS reads.  The
// next 32 pixels are loaded into registers while the current ones feed the
// products.  A workgroup owns all COUT x (TPG taps x CIN) outputs of its tap
// group; its four waves split them 2 x 2 (MW co tiles x NW column tiles each),
// and the waves of tap group 0 with column half 0 also take the bias (a
// product with a B fragment of ones).  Pixels past the split read 0.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int TPG>
struct WgradTile {
  static constexpr int KS = 32;               // pixels per stage
  // LDS row: 72 bytes, so the rows 8 apart that one transposed write touches
  // fall in different banks; fragments are then 8-byte aligned (two 8-byte reads)
  static constexpr int ROW = KS + 4;
  static constexpr int NMT = COUT / 16, NCT = TPG * CIN / 16;
  static constexpr int MW = NMT / 2, NW = NCT / 2;
  static constexpr int UA = (KS / 4) * (COUT / 8);          // staging units of d_out
  static constexpr int UB = (KS / 4) * TPG * (CIN / 8);     // staging units of the input
  static constexpr int ROUNDS = (UA + UB + 255) / 256;
  static constexpr int ROWS = COUT + TPG * CIN;
  static_assert(NMT % 2 == 0 && NCT % 2 == 0 && 9 % TPG == 0, "tile split");
};

// Eight BF16 from an 8-byte aligned LDS address.
FSMI_DEV bf16x8 lds_frag8(const bf16* p) {
  const uint2 lo = *reinterpret_cast<const uint2*>(p), hi = *reinterpret_cast<const uint2*>(p + 4);
  return __builtin_bit_cast(bf16x8, uint4{lo.x, lo.y, hi.x, hi.y});
}

// Transpose four vectors of 8 BF16 channels (pixels 0..3): row k gets channel
// k of the four pixels, as two dwords.
FSMI_DEV void transpose4x8(const bf16x8 (&v)[4], uint2 (&row)[8]) {
  uint32_t x[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint4 u = __builtin_bit_cast(uint4, v[j]);
    x[j][0] = u.x;
    x[j][1] = u.y;
    x[j][2] = u.z;
    x[j][3] = u.w;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    // low halves hold channel 2 d, high halves channel 2 d + 1
    row[2 * d] = uint2{__builtin_amdgcn_perm(x[1][d], x[0][d], 0x05040100u),
                       __builtin_amdgcn_perm(x[3][d], x[2][d], 0x05040100u)};
    row[2 * d + 1] = uint2{__builtin_amdgcn_perm(x[1][d], x[0][d], 0x07060302u),
                           __builtin_amdgcn_perm(x[3][d], x[2][d], 0x07060302u)};
  }
}

template <int CIN, int COUT, int HIN, int TPG>
__global__ __launch_bounds__(256) void k_conv_wgrad(int64_t npix_out, int chunk,
                                                    const bf16* __restrict__ dout,
                                                    const bf16* __restrict__ in,
                                                    float* __restrict__ part) {
  using T = WgradTile<CIN, COUT, TPG>;
  constexpr int HOUT = HIN / 2, NCOL = 9 * CIN + 16;
  constexpr int KS = T::KS, ROW = T::ROW, MW = T::MW, NW = T::NW, ROUNDS = T::ROUNDS;
  constexpr int UA = T::UA, UB = T::UB, QK = KS / 4;
  __shared__ __align__(16) bf16 sL[T::ROWS * ROW];   // rows 0..COUT-1: d_out; then the input
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int i = lane & 15, g = lane >> 4;
  const int s = blockIdx.x, tg = blockIdx.y;
  const int64_t p0 = (int64_t)s * chunk;
  const int64_t p1 = min<int64_t>(p0 + chunk, npix_out);
  const int nstep = (int)((p1 - p0 + KS - 1) / KS);
  const bool bias = tg == 0 && wn == 0;
  floatx4 acc[MW][NW], accb[MW];
#pragma unroll
  for (int mw = 0; mw < MW; ++mw) {
    accb[mw] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nw = 0; nw < NW; ++nw) acc[mw][nw] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  bf16x8 ones;
#pragma unroll
  for (int q = 0; q < 8; ++q) ones[q] = (bf16)1.0f;

  bf16x8 v[ROUNDS][4];
  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const int u = tid + 256 * r;
      if (u < UA) {
        const int pq = u % QK, o = u / QK;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = k0 + 4 * pq + j;
          v[r][j] = p < p1 ? load8(dout + p * COUT + 8 * o) : zero8();
        }
      } else if (u < UA + UB) {
        const int w = u - UA;
        const int pq = w % QK, rest = w / QK;
        const int c8 = rest % (CIN / 8), tap = tg * TPG + rest / (CIN / 8);
        const int ky = tap / 3, kx = tap % 3;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = k0 + 4 * pq + j;
          const int64_t b = p / (HOUT * HOUT);
          const int oy = (int)((p / HOUT) % HOUT), ox = (int)(p % HOUT);
          const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
          const bool ok = p < p1 && iy >= 0 && iy < HIN && ix >= 0 && ix < HIN;
          v[r][j] = ok ? load8(in + ((b * HIN + iy) * HIN + ix) * CIN + 8 * c8) : zero8();
        }
      }
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const int u = tid + 256 * r;
      if (u < UA + UB) {
        int row0, pq;
        if (u < UA) {
          pq = u % QK;
          row0 = 8 * (u / QK);
        } else {
          const int w = u - UA;
          pq = w % QK;
          const int rest = w / QK;
          row0 = COUT + (rest / (CIN / 8)) * CIN + 8 * (rest % (CIN / 8));
        }
        uint2 rows[8];
        transpose4x8(v[r], rows);
#pragma unroll
        for (int k = 0; k < 8; ++k)
          *reinterpret_cast<uint2*>(sL + (row0 + k) * ROW + 4 * pq) = rows[k];
      }
    }
  };

  if (nstep > 0) load_stage(p0);
#pragma unroll 1
  for (int st = 0; st < nstep; ++st) {
    __syncthreads();   // every wave is done reading the previous stage
    store_stage();
    __syncthreads();
    if (st + 1 < nstep) load_stage(p0 + (int64_t)(st + 1) * KS);
    bf16x8 fa[MW];
#pragma unroll
    for (int mw = 0; mw < MW; ++mw)
      fa[mw] = lds_frag8(sL + (16 * (wm * MW + mw) + i) * ROW + 8 * g);
#pragma unroll
    for (int nw = 0; nw < NW; ++nw) {
      const bf16x8 fb = lds_frag8(sL + (COUT + 16 * (wn * NW + nw) + i) * ROW + 8 * g);
#pragma unroll
      for (int mw = 0; mw < MW; ++mw) acc[mw][nw] = mfma(fa[mw], fb, acc[mw][nw]);
    }
    if (bias) {
#pragma unroll
      for (int mw = 0; mw < MW; ++mw) accb[mw] = mfma(fa[mw], ones, accb[mw]);
    }
  }
  // D[4 g + r][i]: co = 16 mt + 4 g + r, column 16 nt + i of the tap group
#pragma unroll
  for (int mw = 0; mw < MW; ++mw) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = 16 * (wm * MW + mw) + 4 * g + r;
      float* row = part + ((int64_t)s * COUT + co) * NCOL;
#pragma unroll
      for (int nw = 0; nw < NW; ++nw) row[tg * TPG * CIN + 16 * (wn * NW + nw) + i] = acc[mw][nw][r];
      if (bias && i == 0) row[9 * CIN] = accb[mw][r];
    }
  }
}

// ---------------------------------------------------------------------------
// grad[W(co, tap, ci)] and grad[b(co)] = sum over splits of the partials, in a
// fixed order: pass 1 sums each run of kRedRun consecutive splits (four lanes
// per output take every fourth split of the run; their four sums are added in
// lane order), pass 2 sums the runs in order.
// ---------------------------------------------------------------------------
constexpr int kRedRun = 32;

template <int CIN, int COUT, bool FIRST>
__global__ __launch_bounds__(256) void k_wgrad_reduce_runs(const float* __restrict__ part, int splits,
                                                           float* __restrict__ runs) {
  constexpr int NCOL = FIRST ? 16 : 9 * CIN + 16;
  constexpr int NW = COUT * 9 * CIN, NOUT = NW + COUT;
  __shared__ float red[4][64];
  const int t = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + t, run = blockIdx.y;
  float sum = 0.0f;
  if (o < NOUT) {
    const int co = o < NW ? o / (9 * CIN) : o - NW;
    const int col = o < NW ? o % (9 * CIN) : 9 * CIN;   // rest = tap CIN + ci, or the bias column
    const int k1 = min(splits, (run + 1) * kRedRun);
    for (int k = run * kRedRun + sl; k < k1; k += 4) sum += part[((int64_t)k * COUT + co) * NCOL + col];
  }
  red[sl][t] = sum;
  __syncthreads();
  if (sl == 0 && o < NOUT) runs[(int64_t)run * NOUT + o] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

template <int CIN, int COUT>
__global__ void k_wgrad_reduce_final(const float* __restrict__ runs, int nrun, float* __restrict__ gW,
                                     float* __restrict__ gb) {
  constexpr int NW = COUT * 9 * CIN, NOUT = NW + COUT;
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= NOUT) return;
  float sum = 0.0f;
  for (int r = 0; r < nrun; ++r) sum += runs[(int64_t)r * NOUT + o];
  if (o < NW)
    gW[o] = sum;
  else
    gb[o - NW] = sum;
}

// ---------------------------------------------------------------------------
// Head: global average pool, FC 128->256, ReLU, FC 256->1 (FP32 VALU).
// kHeadPoses poses per workgroup of 256 threads: thread t is hidden unit t and
// reads its FC1 weight row once for all the workgroup's poses.  Per pose the
// sums run in the same order as one pose at a time would take them.
// ---------------------------------------------------------------------------
constexpr int kHeadPoses = 16;
__global__ __launch_bounds__(256) void k_head_fwd(int64_t n, const bf16* __restrict__ act5,
                                                  const float* __restrict__ P, float* __restrict__ gsave,
                                                  float* __restrict__ hsave, float* __restrict__ ypred) {
  __shared__ float g[kHeadPoses][kFeat];
  __shared__ float red[kHeadPoses][4];
  const int t = threadIdx.x;
  for (int64_t b0 = (int64_t)blockIdx.x * kHeadPoses; b0 < n; b0 += (int64_t)gridDim.x * kHeadPoses) {
    const int nb = (int)min<int64_t>(kHeadPoses, n - b0);
    for (int e = t; e < nb * kFeat; e += 256) {
      const int pb = e / kFeat, c = e - pb * kFeat;
      const int64_t b = b0 + pb;
      float s = 0.0f;
      for (int q = 0; q < 16; ++q) s += (float)act5[(b * 16 + q) * kFeat + c];
      g[pb][c] = s * (1.0f / 16.0f);
      if (gsave) gsave[b * kFeat + c] = g[pb][c];
    }
    __syncthreads();
    float h[kHeadPoses];
    const float bias = P[kC1 + t];
#pragma unroll
    for (int pb = 0; pb < kHeadPoses; ++pb) h[pb] = bias;
    const float* w = P + kF1 + t * kFeat;
    for (int c = 0; c < kFeat; c += 4) {
      const float4 w4 = *reinterpret_cast<const float4*>(w + c);
#pragma unroll
      for (int pb = 0; pb < kHeadPoses; ++pb) {
        h[pb] = fmaf(w4.x, g[pb][c], h[pb]);
        h[pb] = fmaf(w4.y, g[pb][c + 1], h[pb]);
        h[pb] = fmaf(w4.z, g[pb][c + 2], h[pb]);
        h[pb] = fmaf(w4.w, g[pb][c + 3], h[pb]);
      }
    }
    const float f2 = P[kF2 + t];
#pragma unroll
    for (int pb = 0; pb < kHeadPoses; ++pb) {
      const float hp = h[pb] > 0.0f ? h[pb] : 0.0f;
      if (pb < nb && hsave) hsave[(b0 + pb) * kHid + t] = hp;
      float y = f2 * hp;
      y = wave_sum(y);
      if ((t & 63) == 0) red[pb][t >> 6] = y;
    }
    __syncthreads();
    if (t < nb) ypred[b0 + t] = ((red[t][0] + red[t][1]) + (red[t][2] + red[t][3])) + P[kC2];
    __syncthreads();
  }
}

// The regression target of a label (nats): e = exp((label - mean) / scale),
// the standardised label passed through exp so that the squared error weights
// the upper tail (the candidates a ranking keeps) more than the bulk, then
// standardised again, (e - emean) / escale.  Monotone, so the ranking it
// learns is the labels' ranking.  stats = {mean, scale, emean, escale}.
FSMI_DEV float sur_target(double label, const double* stats) {
  return (float)((exp((label - stats[0]) / stats[1]) - stats[2]) / stats[3]);
}

// Head backward for one pose: dy = 2 (y - target) / n; dh = dy F2 [h > 0];
// dg = F1^T dh; d_act5[p][c] = dg[c] / 16 [act5 > 0].
__global__ __launch_bounds__(256) void k_head_bwd(int64_t n, const float* __restrict__ ypred,
                                                  const double* __restrict__ labels,
                                                  const double* __restrict__ stats,
                                                  const float* __restrict__ P,
                                                  const float* __restrict__ hsave,
                                                  const bf16* __restrict__ act5,
                                                  float* __restrict__ dysave,
                                                  float* __restrict__ dhsave,
                                                  bf16* __restrict__ dact5) {
  __shared__ float dh[kHid];
  const int t = threadIdx.x;
  for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
    const float target = sur_target(labels[b], stats);
    const float dy = 2.0f * (ypred[b] - target) / (float)n;
    if (t == 0) dysave[b] = dy;
    const float h = hsave[b * kHid + t];
    const float d = h > 0.0f ? dy * P[kF2 + t] : 0.0f;
    dh[t] = d;
    dhsave[b * kHid + t] = d;
    __syncthreads();
    if (t < kFeat) {
      float s = 0.0f;
      for (int k = 0; k < kHid; ++k) s = fmaf(P[kF1 + k * kFeat + t], dh[k], s);
      const float gs = s * (1.0f / 16.0f);
      for (int q = 0; q < 16; ++q) {
        const int64_t idx = (b * 16 + q) * kFeat + t;
        dact5[idx] = (bf16)((float)act5[idx] > 0.0f ? gs : 0.0f);
      }
    }
    __syncthreads();
  }
}

// Head weight gradients and the loss, each a fixed-order sum over the batch.
// Pass 1: workgroup (kt, j) sums the poses of chunk j, in order, for the rows
// k in [32 kt, 32 kt + 32): dF1[k][c] = sum_b dh[b][k] g[b][c], dc1[k] =
// sum_b dh[b][k], dF2[k] = sum_b dy[b] h[b][k]; the workgroups kt = 0 also
// take dc2 = sum_b dy[b] and the squared error.  The chunk's poses pass
// through LDS 64 at a time.  Pass 2 adds the chunks in order.
constexpr int kHeadOut = kHid * kFeat + 2 * kHid + 2;   // dF1, dc1, dF2, dc2, loss
constexpr int kHeadMaxChunks = 64;

__global__ __launch_bounds__(256) void k_head_wgrad_part(
    int64_t n, int64_t chunk, const float* __restrict__ gsave, const float* __restrict__ hsave,
    const float* __restrict__ dysave, const float* __restrict__ dhsave,
    const float* __restrict__ ypred, const double* __restrict__ labels,
    const double* __restrict__ stats, float* __restrict__ part) {
  __shared__ float sdh[64][32], sh[64][32], sg[64][kFeat], sdy[64], se[64];
  const int t = threadIdx.x, kt = blockIdx.x, j = blockIdx.y;
  const int64_t b0 = (int64_t)j * chunk, b1 = min<int64_t>(b0 + chunk, n);
  const int kp = 2 * (t / 16), c0 = t % 16;   // rows 32 kt + kp + {0, 1}, columns c0 + 16 q
  float acc[2][8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[0][q] = acc[1][q] = 0.0f;
  float aux = 0.0f;   // t < 32: dc1; t < 64: dF2; with kt = 0, t = 64: dc2, t = 65: squared error
  for (int64_t s0 = b0; s0 < b1; s0 += 64) {
    const int nb = (int)min<int64_t>(64, b1 - s0);
    __syncthreads();   // the previous poses are consumed
    for (int e = t; e < 64 * 32; e += 256) {
      const int bb = e / 32, kk = e % 32;
      const bool ok = bb < nb;
      sdh[bb][kk] = ok ? dhsave[(s0 + bb) * kHid + 32 * kt + kk] : 0.0f;
      sh[bb][kk] = ok ? hsave[(s0 + bb) * kHid + 32 * kt + kk] : 0.0f;
    }
    for (int e = t; e < 64 * kFeat; e += 256) {
      const int bb = e / kFeat, c = e % kFeat;
      sg[bb][c] = bb < nb ? gsave[(s0 + bb) * kFeat + c] : 0.0f;
    }
    if (t < 64) {
      const bool ok = t < nb;
      sdy[t] = ok ? dysave[s0 + t] : 0.0f;
      float ev = 0.0f;
      if (ok && kt == 0) ev = ypred[s0 + t] - sur_target(labels[s0 + t], stats);
      se[t] = ev;
    }
    __syncthreads();
    for (int bb = 0; bb < nb; ++bb) {
      const float d0 = sdh[bb][kp], d1 = sdh[bb][kp + 1];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float gv = sg[bb][c0 + 16 * q];
        acc[0][q] = fmaf(d0, gv, acc[0][q]);
        acc[1][q] = fmaf(d1, gv, acc[1][q]);
      }
      if (t < 32)
        aux += sdh[bb][t];
      else if (t < 64)
        aux = fmaf(sdy[bb], sh[bb][t - 32], aux);
      else if (t == 64)
        aux += sdy[bb];
      else if (t == 65)
        aux = fmaf(se[bb], se[bb], aux);
    }
  }
  float* out = part + (int64_t)j * kHeadOut;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 8; ++q) out[(32 * kt + kp + r) * kFeat + c0 + 16 * q] = acc[r][q];
  if (t < 32)
    out[kHid * kFeat + 32 * kt + t] = aux;
  else if (t < 64)
    out[kHid * kFeat + kHid + 32 * kt + t - 32] = aux;
  else if (kt == 0 && t < 66)
    out[kHid * kFeat + 2 * kHid + (t - 64)] = aux;
}

__global__ __launch_bounds__(256) void k_head_wgrad_final(int64_t n, int nchunk,
                                                          const float* __restrict__ part,
                                                          float* __restrict__ G,
                                                          float* __restrict__ loss) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= kHeadOut) return;
  float s = 0.0f;
  for (int j = 0; j < nchunk; ++j) s += part[(int64_t)j * kHeadOut + o];
  constexpr int nF1 = kHid * kFeat;
  if (o < nF1)
    G[kF1 + o] = s;
  else if (o < nF1 + kHid)
    G[kC1 + (o - nF1)] = s;
  else if (o < nF1 + 2 * kHid)
    G[kF2 + (o - nF1 - kHid)] = s;
  else if (o == nF1 + 2 * kHid)
    G[kC2] = s;
  else if (loss)
    *loss = s / (float)n;
}

// ---------------------------------------------------------------------------
// Parameters: init, BF16 copies, Adam
// ---------------------------------------------------------------------------
FSMI_DEV uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Kaiming-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)) (sqrt(3/fan_in) for the
// output layer), zero biases, zero Adam moments.  Draws: splitmix64(seed ^ index).
__global__ void k_sur_init(uint64_t seed, float* P, float* M, float* V) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNumParams) return;
  float bound = 0.0f;
#pragma unroll
  for (int l = 0; l < 5; ++l)
    if (t >= w_off(l) && t < b_off(l)) bound = sqrtf(6.0f / (9.0f * kL[l].cin));
  if (t >= kF1 && t < kC1) bound = sqrtf(6.0f / kFeat);
  if (t >= kF2 && t < kC2) bound = sqrtf(3.0f / kHid);
  const uint64_t r = splitmix64(seed ^ ((uint64_t)t * 0x632BE59BD9B4E019ull));
  const float u = (float)(r >> 40) * (1.0f / 16777216.0f);   // [0, 1)
  P[t] = bound * (2.0f * u - 1.0f);
  M[t] = 0.0f;
  V[t] = 0.0f;
}

__global__ void k_sur_cast(const float* __restrict__ P, bf16* __restrict__ Wbf,
                           bf16* __restrict__ Wt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kWbfTotal) return;
  int l = 0;
  while (l < 4 && t >= wbf_off(l + 1)) ++l;
  const int e = t - wbf_off(l);
  const int cin = kL[l].cin, cout = kL[l].cout;
  const int co = e / (9 * cin), rest = e % (9 * cin), tap = rest / cin, ci = rest % cin;
  const bf16 v = (bf16)P[w_off(l) + e];
  Wbf[t] = v;
  Wt[wbf_off(l) + (tap * cin + ci) * cout + co] = v;
}

__global__ void k_adam(float* P, const float* G, float* M, float* V, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNumParams) return;
  const float g = G[t];
  const float m = b1 * M[t] + (1.0f - b1) * g;
  const float v = b2 * V[t] + (1.0f - b2) * g * g;
  M[t] = m;
  V[t] = v;
  P[t] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Label statistics: mean and standard deviation of n FP64 labels (two-pass, one
// workgroup, fixed order).
__global__ void k_label_stats(int64_t n, const double* labels, double* stats) {
  __shared__ double red[16];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < n; i += blockDim.x) s += labels[i];
  s = wave_sum(s);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  double mean = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) mean += red[k];
  mean /= (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t i = t; i < n; i += blockDim.x) q += (labels[i] - mean) * (labels[i] - mean);
  q = wave_sum(q);
  if ((t & 63) == 0) red[t >> 6] = q;
  __syncthreads();
  double v = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v += red[k];
  v = sqrt(v / (double)n);
  const double scale = v > 0.0 ? v : 1.0;
  __syncthreads();
  // mean and standard deviation of e = exp((label - mean) / scale)
  double se = 0.0;
  for (int64_t i = t; i < n; i += blockDim.x) se += exp((labels[i] - mean) / scale);
  se = wave_sum(se);
  if ((t & 63) == 0) red[t >> 6] = se;
  __syncthreads();
  double emean = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) emean += red[k];
  emean /= (double)n;
  __syncthreads();
  double qe = 0.0;
  for (int64_t i = t; i < n; i += blockDim.x) {
    const double d = exp((labels[i] - mean) / scale) - emean;
    qe += d * d;
  }
  qe = wave_sum(qe);
  if ((t & 63) == 0) red[t >> 6] = qe;
  __syncthreads();
  if (t == 0) {
    double ve = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) ve += red[k];
    ve = sqrt(ve / (double)n);
    stats[0] = mean;
    stats[1] = scale;
    stats[2] = emean;
    stats[3] = ve > 0.0 ? ve : 1.0;
  }
}

// Predictions in nats, the target's inverse: mean + scale ln(y escale + emean)
// (the logarithm's argument clamped to 1e-6 from below: a prediction at or
// under the exponential's range reads as 13.8 scales under the mean).
__global__ void k_destandardise(int64_t n, const float* y, const double* stats, float* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const double e = (double)y[i] * stats[3] + stats[2];
    out[i] = (float)(log(fmax(e, 1e-6)) * stats[1] + stats[0]);
  }
}

// One 16x16x32 product through the matrix core, A and B row-major (diagnostic).
__global__ void k_mfma_probe(const bf16* A, const bf16* B, float* D) {
  const int l = threadIdx.x, i = l & 15, g = l >> 4;
  bf16x8 a, b;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = A[i * 32 + 8 * g + q];
    b[q] = B[(8 * g + q) * 16 + i];
  }
  floatx4 d = mfma(a, b, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
  for (int r = 0; r < 4; ++r) D[(4 * g + r) * 16 + i] = d[r];
}

// ---------------------------------------------------------------------------
// Top-k: bitonic sort of (key, index) pairs, keys descending, ties by index.
// ---------------------------------------------------------------------------
__global__ void k_topk_fill(int64_t n, int64_t npow2, const float* pred, float* key, int32_t* idx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npow2) return;
  const float v = i < n ? pred[i] : -INFINITY;
  key[i] = (v == v) ? v : -INFINITY;   // NaN sorts last
  idx[i] = (int32_t)i;
}

__global__ void k_bitonic_step(int64_t npow2, int64_t j, int64_t k, float* key, int32_t* idx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npow2) return;
  const int64_t p = i ^ j;
  if (p <= i) return;
  const float a = key[i], b = key[p];
  const int32_t ia = idx[i], ib = idx[p];
  // "a before b" in descending order with ties by ascending index
  const bool a_first = (a > b) || (a == b && ia < ib);
  const bool up = (i & k) == 0;
  if (up != a_first) {
    key[i] = b;
    key[p] = a;
    idx[i] = ib;
    idx[p] = ia;
  }
}

__global__ void k_gather_poses(int k, const int32_t* idx, const double* poses, double* out,
                               int32_t* idx_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k) return;
  const int32_t j = idx[t];
  for (int q = 0; q < 4; ++q) out[4 * t + q] = poses[4 * (int64_t)j + q];
  if (idx_out) idx_out[t] = j;
}

}  // namespace fsmi

// ===========================================================================
// Host side
// ===========================================================================
struct fsmi_sur_s {
  fsmi_ctx ctx = nullptr;
  int max_batch = 0;
  int step = 0;
  float* P = nullptr;       // master weights [kNumParams]
  float* G = nullptr;       // gradients
  float* M = nullptr;       // Adam first moment
  float* V = nullptr;       // Adam second moment
  fsmi::bf16* Wbf = nullptr;
  fsmi::bf16* Wt = nullptr;
  double* stats = nullptr;  // label mean, scale
  fsmi::bf16* act[6] = {};  // act[1..5]
  fsmi::bf16* dact[6] = {}; // gradients of act[1..5]
  float* gsave = nullptr;
  float* hsave = nullptr;
  float* dysave = nullptr;
  float* dhsave = nullptr;
  float* ypred = nullptr;
  float* part = nullptr;    // weight-gradient partials
  float* runs = nullptr;    // their sums over runs of splits
  float* hpart = nullptr;   // head-gradient partials per chunk of poses
  size_t part_floats = 0;
  float* loss = nullptr;
  int stride = 1;            // cell stride of the patch
  void* sign[5] = {};            // sign[l]: ReLU sign words of act[l], l = 1..4 (training)
  float* pooled = nullptr;   // block means of the last map (stride > 1)
  size_t pooled_elems = 0;
  fsmi::PatchOrigin* porg = nullptr;   // patch origins of the batch's poses
};

namespace fsmi {

// Weight-gradient splits per layer, at most, and taps per workgroup of the
// weight-gradient kernel (conv1's weight gradient is taken inside conv2's
// input-gradient pass, in wg1_splits(nb) splits).  A layer's splits are a
// fixed count rather than a fixed length: the split length follows the batch
// (wg_chunk), so the grid, kWgSplits[l] x 9 / kWgTpg[l] workgroups, and the
// partial sums stay the same size at any batch.
static constexpr int kWgSplits[5] = {0, 512, 256, 128, 32};
static constexpr int kWgTpg[5] = {0, 9, 3, 3, 1};
constexpr int kWgStage = 32;   // pixels per stage of k_conv_wgrad (WgradTile::KS)

// Split length for npix output pixels: a multiple of the stage, at least one
// stage, and long enough for at most kWgSplits[l] splits.
static int64_t wg_chunk(int l, int64_t npix) {
  const int64_t per = (npix + kWgSplits[l] - 1) / kWgSplits[l];
  return std::max<int64_t>(kWgStage, (per + kWgStage - 1) / kWgStage * kWgStage);
}

// Splits (workgroups) of conv2's input-gradient pass with conv1's weight
// gradient fused in, for nb poses, and the tiles each takes.  With n tiles
// and W = kWg1PerCu x num_cu, the splits are ceil(n / ceil(n / W)) <= min(n,
// W); that count is not monotone in n (n = W gives W, n = W + 1 gives about
// W / 2), so the partial buffer is sized by wg1_max_splits, min(n, W) at the
// largest batch.
static int64_t wg1_tiles(int64_t nb) {
  constexpr int tq = 16 * dgrad_mt<kL[1].cin, kL[1].cout, kL[1].hin>();
  return nb * (kL[1].hin / 2) * (kL[1].hin / 2) / tq;
}
static int64_t wg1_splits(int64_t nb, int num_cu, int* tiles_per_wg) {
  const int64_t n_tiles = wg1_tiles(nb);
  const int64_t w = (int64_t)kWg1PerCu * num_cu;
  const int64_t per = std::max<int64_t>(1, (n_tiles + w - 1) / w);
  *tiles_per_wg = (int)per;
  return (n_tiles + per - 1) / per;
}
static int64_t wg1_max_splits(int64_t max_batch, int num_cu) {
  return std::min<int64_t>(wg1_tiles(max_batch), (int64_t)kWg1PerCu * num_cu);
}

static size_t act_elems(int l, int B) {   // elements of act[l] (output of conv l-1... l = 1..5)
  const int h = kL[l - 1].hin / 2;
  return (size_t)B * h * h * kL[l - 1].cout;
}

static hipError_t sur_alloc(fsmi_sur net) {
  hipError_t e;
#define ALLOC(ptr, bytes)                                  \
  do {                                                     \
    e = hipMalloc((void**)&(ptr), (bytes));                \
    if (e != hipSuccess) return e;                         \
  } while (0)
  ALLOC(net->P, sizeof(float) * kNumParams);
  ALLOC(net->G, sizeof(float) * kNumParams);
  ALLOC(net->M, sizeof(float) * kNumParams);
  ALLOC(net->V, sizeof(float) * kNumParams);
  ALLOC(net->Wbf, sizeof(bf16) * kWbfTotal);
  ALLOC(net->Wt, sizeof(bf16) * kWbfTotal);
  ALLOC(net->stats, 16 * sizeof(double));
  const int B = net->max_batch;
  for (int l = 1; l <= 5; ++l) {
    ALLOC(net->act[l], sizeof(bf16) * act_elems(l, B));
    if (l >= 2) ALLOC(net->dact[l], sizeof(bf16) * act_elems(l, B));   // conv1's d_out stays on chip
    if (l <= 4) ALLOC(net->sign[l], act_elems(l, B) / 8);   // one bit per channel
  }
  ALLOC(net->gsave, sizeof(float) * (size_t)B * kFeat);
  ALLOC(net->hsave, sizeof(float) * (size_t)B * kHid);
  ALLOC(net->dysave, sizeof(float) * (size_t)B);
  ALLOC(net->dhsave, sizeof(float) * (size_t)B * kHid);
  ALLOC(net->ypred, sizeof(float) * (size_t)B);
  ALLOC(net->porg, sizeof(PatchOrigin) * (size_t)B);
  size_t mx = 0, mr = 0;
  for (int l = 0; l < 5; ++l) {
    const int hout = kL[l].hin / 2;
    const size_t npix = (size_t)B * hout * hout;
    // conv1's weight gradient is taken inside conv2's input-gradient pass
    const size_t splits =
        l == 0 ? (size_t)wg1_max_splits(B, net->ctx->num_cu) : (size_t)kWgSplits[l];
    const size_t ncol = l == 0 ? 16 : 9 * (size_t)kL[l].cin + 16;
    const size_t nout = (size_t)kL[l].cout * (9 * kL[l].cin + 1);
    mx = std::max(mx, splits * kL[l].cout * ncol);
    mr = std::max(mr, (splits + kRedRun - 1) / kRedRun * nout);
  }
  net->part_floats = mx;
  ALLOC(net->part, sizeof(float) * mx);
  ALLOC(net->runs, sizeof(float) * mr);
  ALLOC(net->hpart, sizeof(float) * (size_t)kHeadMaxChunks * kHeadOut);
  ALLOC(net->loss, sizeof(float) * 4);
#undef ALLOC
  return hipSuccess;
}

static void sur_free(fsmi_sur net) {
  void* ps[] = {net->P, net->G, net->M, net->V, net->Wbf, net->Wt, net->stats, net->gsave,
                net->hsave, net->dysave, net->dhsave, net->ypred, net->part, net->runs, net->hpart, net->loss,
                net->porg};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (net->pooled) (void)hipFree(net->pooled);
  for (int l = 1; l <= 4; ++l)
    if (net->sign[l]) (void)hipFree(net->sign[l]);
  for (int l = 1; l <= 5; ++l) {
    if (net->act[l]) (void)hipFree(net->act[l]);
    if (net->dact[l]) (void)hipFree(net->dact[l]);
  }
}

// The first layer's input for `map`: the map itself, or (stride > 1) its block
// means, recomputed on the net's stream for this call.
static hipError_t make_src(fsmi_sur net, const fsmi_map* map, const double* poses, PatchSrc* src) {
  const int s = net->stride;
  if (s == 1) {
    *src = PatchSrc{map->occ, map->dims[0], map->dims[1], poses, 1};
    return hipSuccess;
  }
  const int64_t X = map->dims[0], Y = map->dims[1];
  const int64_t Xc = (X + s - 1) / s, Yc = (Y + s - 1) / s;
  if ((size_t)(Xc * Yc) > net->pooled_elems) {
    if (net->pooled) {
      hipError_t e = hipStreamSynchronize(net->ctx->stream);
      if (e != hipSuccess) return e;
      (void)hipFree(net->pooled);
      net->pooled = nullptr;
      net->pooled_elems = 0;
    }
    hipError_t e = hipMalloc((void**)&net->pooled, sizeof(float) * (size_t)(Xc * Yc));
    if (e != hipSuccess) return e;
    net->pooled_elems = (size_t)(Xc * Yc);
  }
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((Xc * Yc + 255) / 256, 4096));
  hipLaunchKernelGGL(k_pool_map, dim3(grid), dim3(256), 0, net->ctx->stream, map->occ, X, Y, s, Xc,
                     Yc, net->pooled);
  *src = PatchSrc{net->pooled, Xc, Yc, poses, s};
  return hipGetLastError();
}

static hipError_t cast_weights(fsmi_sur net) {
  hipLaunchKernelGGL(k_sur_cast, dim3((kWbfTotal + 255) / 256), dim3(256), 0, net->ctx->stream,
                     net->P, net->Wbf, net->Wt);
  return hipGetLastError();
}

// Layers after the first two (conv1 and conv2 run fused in k_conv12_fwd).
template <int L>
static void conv_fwd(fsmi_sur net, int64_t nb, bool save) {
  constexpr LayerDims d = kL[L];
  static_assert(L >= 2, "conv1 and conv2 run in k_conv12_fwd");
  if constexpr (L == 2) {
    static_assert(d.cin == 64 && d.cout == 64 && d.hin == 32, "k_conv3_rows is written for conv3");
    const int64_t units = nb * 4;
    const int grid = (int)std::min<int64_t>((units + kC3Waves - 1) / kC3Waves, (int64_t)net->ctx->num_cu * 2);
    hipLaunchKernelGGL(k_conv3_rows, dim3(grid), dim3(64 * kC3Waves), 0, net->ctx->stream, units,
                       net->act[L], net->Wbf + wbf_off(L), net->P + b_off(L), net->act[L + 1],
                       save ? (uint16_t*)net->sign[L + 1] : nullptr);
    return;
  }
  if constexpr (L == 3) {
    static_assert(d.cin == 64 && d.cout == 128 && d.hin == 16, "k_conv4_rows is written for conv4");
    const int64_t units = nb * 4;
    const int grid = (int)std::min<int64_t>((units + kC4Waves - 1) / kC4Waves, (int64_t)net->ctx->num_cu);
    hipLaunchKernelGGL(k_conv4_rows, dim3(grid), dim3(64 * kC4Waves), 0,
                       net->ctx->stream, units, net->act[L], net->Wbf + wbf_off(L), net->P + b_off(L),
                       net->act[L + 1], save ? (uint32_t*)net->sign[L + 1] : nullptr);
    return;
  }
  if constexpr (L == 4) {
    static_assert(d.cin == 128 && d.cout == 128 && d.hin == 8, "k_conv5_rows is written for conv5");
    const int grid = 2 * (int)std::min<int64_t>((nb + kC5Waves - 1) / kC5Waves, (int64_t)net->ctx->num_cu / 2);
    (void)save;   // act5 has no sign words
    hipLaunchKernelGGL(k_conv5_rows, dim3(grid), dim3(64 * kC5Waves), 0, net->ctx->stream, nb,
                       net->act[L], net->Wbf + wbf_off(L), net->P + b_off(L), net->act[L + 1]);
    return;
  }
  static_assert(L <= 4, "five conv layers");
}

// Forward of nb (<= max_batch) poses; predictions (standardised) in ypred.
// Sets src.org to the batch's patch origins, computed here.
static hipError_t sur_fwd_batch(fsmi_sur net, int64_t nb, PatchSrc& src, bool save) {
  static_assert(kL[0].cout == 32 && kL[1].cin == 32 && kL[1].cout == 64 && kL[1].hin == 64,
                "k_conv12_fwd is written for conv1 1->32 on 128^2 and conv2 32->64");
  hipLaunchKernelGGL(k_patch_origin, dim3((unsigned)std::min<int64_t>((nb + 255) / 256, 1024)), dim3(256),
                     0, net->ctx->stream, nb, src, net->porg);
  src.org = net->porg;
  const int64_t n_tiles = nb * 16;
  const int grid12 = (int)std::min<int64_t>(n_tiles, (int64_t)net->ctx->num_cu * 2);
  if (save)   // training keeps conv1's activations and the sign words
    hipLaunchKernelGGL(k_conv12_fwd<true>, dim3(grid12), dim3(256), 0, net->ctx->stream, n_tiles,
                       src, net->Wbf + wbf_off(0), net->P + b_off(0), net->Wbf + wbf_off(1),
                       net->P + b_off(1), net->act[2], net->act[1],
                       reinterpret_cast<uint8_t*>(net->sign[1]),
                       reinterpret_cast<uint16_t*>(net->sign[2]));
  else
    hipLaunchKernelGGL(k_conv12_fwd<false>, dim3(grid12), dim3(256), 0, net->ctx->stream, n_tiles,
                       src, net->Wbf + wbf_off(0), net->P + b_off(0), net->Wbf + wbf_off(1),
                       net->P + b_off(1), net->act[2], nullptr, nullptr, nullptr);
  conv_fwd<2>(net, nb, save);
  conv_fwd<3>(net, nb, save);
  conv_fwd<4>(net, nb, save);
  const int grid = (int)std::min<int64_t>((nb + kHeadPoses - 1) / kHeadPoses, 65535);
  hipLaunchKernelGGL(k_head_fwd, dim3(grid), dim3(256), 0, net->ctx->stream, nb, net->act[5], net->P,
                     save ? net->gsave : nullptr, save ? net->hsave : nullptr, net->ypred);
  return hipGetLastError();
}

template <int L>
static void conv_dgrad(fsmi_sur net, int64_t nb) {
  constexpr LayerDims d = kL[L];
  static_assert(L >= 2, "conv2's pass runs fused with conv1's weight gradient");
  constexpr int mt = dgrad_mt<d.cin, d.cout, d.hin>();
  const int64_t nq = nb * (d.hin / 2) * (d.hin / 2);   // a multiple of 16
  hipLaunchKernelGGL((k_conv_dgrad<d.cin, d.cout, d.hin, false>),
                     dim3((unsigned)((nq + 16 * mt - 1) / (16 * mt))), dim3(256), 0, net->ctx->stream,
                     nq, 1, net->dact[L + 1], net->Wt + wbf_off(L), net->act[L],
                     net->sign[L], net->dact[L], PatchSrc{}, nullptr);
}

// conv2's input gradient and conv1's weight gradient (k_conv_dgrad with WG1),
// then conv1's partials summed in fixed order.
static void conv2_dgrad_conv1_wgrad(fsmi_sur net, int64_t nb, PatchSrc src) {
  constexpr LayerDims d1 = kL[1], d0 = kL[0];
  hipStream_t st = net->ctx->stream;
  const int64_t nq = nb * (d1.hin / 2) * (d1.hin / 2);
  int per = 1;
  const int splits = (int)wg1_splits(nb, net->ctx->num_cu, &per);
  hipLaunchKernelGGL((k_conv_dgrad<d1.cin, d1.cout, d1.hin, true>), dim3(splits), dim3(256), 0, st, nq,
                     per, net->dact[2], net->Wt + wbf_off(1), net->act[1], net->sign[1], nullptr,
                     src, net->part);
  constexpr int nout = d0.cout * 9 * d0.cin + d0.cout;
  const int nrun = (splits + kRedRun - 1) / kRedRun;
  hipLaunchKernelGGL((k_wgrad_reduce_runs<d0.cin, d0.cout, true>), dim3((nout + 63) / 64, nrun),
                     dim3(256), 0, st, net->part, splits, net->runs);
  hipLaunchKernelGGL((k_wgrad_reduce_final<d0.cin, d0.cout>), dim3((nout + 255) / 256), dim3(256), 0, st,
                     net->runs, nrun, net->G + w_off(0), net->G + b_off(0));
}

template <int L>
static void conv_wgrad(fsmi_sur net, int64_t nb) {
  constexpr LayerDims d = kL[L];
  static_assert(L >= 1, "conv1's weight gradient is taken in conv2_dgrad_conv1_wgrad");
  hipStream_t st = net->ctx->stream;
  const int64_t npix = nb * (d.hin / 2) * (d.hin / 2);
  static_assert(WgradTile<d.cin, d.cout, kWgTpg[L]>::KS == kWgStage, "split lengths are whole stages");
  const int chunk = (int)wg_chunk(L, npix);   // <= kWgSplits[L] splits
  const int splits = (int)((npix + chunk - 1) / chunk);
  constexpr int tpg = kWgTpg[L];
  hipLaunchKernelGGL((k_conv_wgrad<d.cin, d.cout, d.hin, tpg>), dim3(splits, 9 / tpg), dim3(256), 0,
                     st, npix, chunk, net->dact[L + 1], net->act[L], net->part);
  constexpr int nout = d.cout * 9 * d.cin + d.cout;
  const int nrun = (splits + kRedRun - 1) / kRedRun;
  hipLaunchKernelGGL((k_wgrad_reduce_runs<d.cin, d.cout, false>), dim3((nout + 63) / 64, nrun),
                     dim3(256), 0, st, net->part, splits, net->runs);
  hipLaunchKernelGGL((k_wgrad_reduce_final<d.cin, d.cout>), dim3((nout + 255) / 256), dim3(256), 0, st,
                     net->runs, nrun, net->G + w_off(L), net->G + b_off(L));
}

}  // namespace fsmi

using namespace fsmi;

extern "C" {

int64_t fsmi_sur_num_params(void) { return kNumParams; }

fsmi_status fsmi_sur_create(fsmi_ctx ctx, fsmi_sur* out, uint64_t seed, int32_t max_batch,
                            int32_t patch_stride) {
  if (!ctx || !out || max_batch <= 0 || max_batch > 65536 || patch_stride < 1 || patch_stride > 64)
    return FSMI_E_INVAL;
  *out = nullptr;
  (void)hipSetDevice(ctx->device);
  fsmi_sur net = new fsmi_sur_s();
  net->ctx = ctx;
  net->max_batch = max_batch;
  net->stride = patch_stride;
  if (sur_alloc(net) != hipSuccess) {
    sur_free(net);
    delete net;
    return FSMI_E_NOMEM;
  }
  hipLaunchKernelGGL(k_sur_init, dim3((kNumParams + 255) / 256), dim3(256), 0, ctx->stream, seed,
                     net->P, net->M, net->V);
  const double st[4] = {0.0, 1.0, 0.0, 1.0};
  (void)hipMemcpy(net->stats, st, sizeof(st), hipMemcpyHostToDevice);
  if (cast_weights(net) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    sur_free(net);
    delete net;
    return FSMI_E_DEVICE;
  }
  *out = net;
  return FSMI_OK;
}

void fsmi_sur_destroy(fsmi_sur net) {
  if (!net) return;
  (void)hipStreamSynchronize(net->ctx->stream);
  sur_free(net);
  delete net;
}

fsmi_status fsmi_sur_fit_label_stats(fsmi_sur net, int64_t n, const double* labels) {
  if (!net || n <= 0 || !labels) return FSMI_E_INVAL;
  hipLaunchKernelGGL(k_label_stats, dim3(1), dim3(1024), 0, net->ctx->stream, n, labels, net->stats);
  return hipGetLastError() == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

static bool sur_map_ok(fsmi_sur net, const fsmi_map* map) {
  return net && map && map->occ && map->ndim == 2 && map->dims[0] > 0 && map->dims[1] > 0;
}

fsmi_status fsmi_sur_forward(fsmi_sur net, const fsmi_map* map, int64_t n, const double* poses,
                             float* pred) {
  if (!sur_map_ok(net, map) || n < 0 || (n > 0 && (!poses || !pred))) return FSMI_E_INVAL;
  (void)hipSetDevice(net->ctx->device);
  if (n == 0) return FSMI_OK;
  PatchSrc src0;
  const hipError_t e = make_src(net, map, poses, &src0);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? FSMI_E_NOMEM : FSMI_E_DEVICE;
  for (int64_t s = 0; s < n; s += net->max_batch) {
    const int64_t nb = std::min<int64_t>(net->max_batch, n - s);
    PatchSrc src = src0;
    src.poses = poses + 4 * s;
    if (sur_fwd_batch(net, nb, src, false) != hipSuccess) return FSMI_E_DEVICE;
    hipLaunchKernelGGL(k_destandardise, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0,
                       net->ctx->stream, nb, net->ypred, net->stats, pred + s);
  }
  return hipGetLastError() == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_sur_backward(fsmi_sur net, const fsmi_map* map, int64_t n, const double* poses,
                              const double* labels, float* loss) {
  if (!sur_map_ok(net, map) || n <= 0 || n > net->max_batch || !poses || !labels)
    return FSMI_E_INVAL;
  (void)hipSetDevice(net->ctx->device);
  PatchSrc src;
  hipError_t e = make_src(net, map, poses, &src);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? FSMI_E_NOMEM : FSMI_E_DEVICE;
  if (sur_fwd_batch(net, n, src, true) != hipSuccess) return FSMI_E_DEVICE;
  hipStream_t st = net->ctx->stream;
  const int grid = (int)std::min<int64_t>(n, 65535);
  hipLaunchKernelGGL(k_head_bwd, dim3(grid), dim3(256), 0, st, n, net->ypred, labels, net->stats,
                     net->P, net->hsave, net->act[5], net->dysave, net->dhsave, net->dact[5]);
  {
    // chunks of a multiple of 64 poses, at most kHeadMaxChunks of them
    const int64_t per = (n + kHeadMaxChunks - 1) / kHeadMaxChunks;
    const int64_t chunk = std::max<int64_t>(64, (per + 63) / 64 * 64);
    const int nchunk = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_head_wgrad_part, dim3(kHid / 32, nchunk), dim3(256), 0, st, n, chunk,
                       net->gsave, net->hsave, net->dysave, net->dhsave, net->ypred, labels,
                       net->stats, net->hpart);
    hipLaunchKernelGGL(k_head_wgrad_final, dim3((kHeadOut + 255) / 256), dim3(256), 0, st, n, nchunk,
                       net->hpart, net->G, loss ? loss : net->loss);
  }
  conv_wgrad<4>(net, n);
  conv_dgrad<4>(net, n);
  conv_wgrad<3>(net, n);
  conv_dgrad<3>(net, n);
  conv_wgrad<2>(net, n);
  conv_dgrad<2>(net, n);
  conv_wgrad<1>(net, n);
  conv2_dgrad_conv1_wgrad(net, n, src);
  return hipGetLastError() == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_sur_adam_step(fsmi_sur net, float lr, float b1, float b2, float eps) {
  if (!net || !(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
    return FSMI_E_INVAL;
  net->step += 1;
  const float c1 = 1.0f - powf(b1, (float)net->step), c2 = 1.0f - powf(b2, (float)net->step);
  hipLaunchKernelGGL(k_adam, dim3((kNumParams + 255) / 256), dim3(256), 0, net->ctx->stream, net->P,
                     net->G, net->M, net->V, lr, b1, b2, eps, c1, c2);
  return cast_weights(net) == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_sur_get_params(fsmi_sur net, float* dst) {
  if (!net || !dst) return FSMI_E_INVAL;
  return hipMemcpyAsync(dst, net->P, sizeof(float) * kNumParams, hipMemcpyDeviceToDevice,
                        net->ctx->stream) == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_sur_set_params(fsmi_sur net, const float* src) {
  if (!net || !src) return FSMI_E_INVAL;
  if (hipMemcpyAsync(net->P, src, sizeof(float) * kNumParams, hipMemcpyDeviceToDevice,
                     net->ctx->stream) != hipSuccess)
    return FSMI_E_DEVICE;
  return cast_weights(net) == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_sur_get_grads(fsmi_sur net, float* dst) {
  if (!net || !dst) return FSMI_E_INVAL;
  return hipMemcpyAsync(dst, net->G, sizeof(float) * kNumParams, hipMemcpyDeviceToDevice,
                        net->ctx->stream) == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_sur_get_label_stats(fsmi_sur net, double* host_stats) {
  if (!net || !host_stats) return FSMI_E_INVAL;
  return hipMemcpy(host_stats, net->stats, 4 * sizeof(double), hipMemcpyDeviceToHost) ==
                 hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

// Checkpoint: magic, step, label stats, master weights, Adam moments (all host order).
fsmi_status fsmi_sur_save(fsmi_sur net, const char* path) {
  if (!net || !path) return FSMI_E_INVAL;
  if (hipStreamSynchronize(net->ctx->stream) != hipSuccess) return FSMI_E_DEVICE;
  std::vector<float> buf(3 * (size_t)kNumParams);
  double st[4];
  if (hipMemcpy(buf.data(), net->P, sizeof(float) * kNumParams, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(buf.data() + kNumParams, net->M, sizeof(float) * kNumParams, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(buf.data() + 2 * kNumParams, net->V, sizeof(float) * kNumParams, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(st, net->stats, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return FSMI_E_DEVICE;
  FILE* f = fopen(path, "wb");
  if (!f) return FSMI_E_INVAL;
  const uint32_t hdr[5] = {0x46534D49u, 3u, (uint32_t)net->step, (uint32_t)kNumParams,
                           (uint32_t)net->stride};
  bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(st, sizeof(st), 1, f) == 1 &&
            fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? FSMI_OK : FSMI_E_INVAL;
}

fsmi_status fsmi_sur_load(fsmi_sur net, const char* path) {
  if (!net || !path) return FSMI_E_INVAL;
  FILE* f = fopen(path, "rb");
  if (!f) return FSMI_E_INVAL;
  uint32_t hdr[5];
  double st[4];
  std::vector<float> buf(3 * (size_t)kNumParams);
  bool ok = fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 0x46534D49u && hdr[1] == 3u &&
            hdr[3] == (uint32_t)kNumParams && hdr[4] >= 1u && hdr[4] <= 64u &&
            fread(st, sizeof(st), 1, f) == 1 &&
            fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  fclose(f);
  if (!ok) return FSMI_E_INVAL;
  net->step = (int)hdr[2];
  net->stride = (int)hdr[4];
  if (hipMemcpy(net->P, buf.data(), sizeof(float) * kNumParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->M, buf.data() + kNumParams, sizeof(float) * kNumParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->V, buf.data() + 2 * kNumParams, sizeof(float) * kNumParams, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->stats, st, sizeof(st), hipMemcpyHostToDevice) != hipSuccess)
    return FSMI_E_DEVICE;
  return cast_weights(net) == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_probe_mfma(fsmi_ctx ctx, const void* A, const void* B, float* D) {
  if (!ctx || !A || !B || !D) return FSMI_E_INVAL;
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, ctx->stream, (const bf16*)A, (const bf16*)B, D);
  return hipGetLastError() == hipSuccess ? FSMI_OK : FSMI_E_DEVICE;
}

fsmi_status fsmi_rank_poses(fsmi_ctx ctx, const fsmi_params* params, fsmi_sur net,
                            const fsmi_map* map, int64_t n_poses, const double* poses,
                            int64_t n_beams, const double* beam_dir, double sigma, double max_range,
                            int32_t k, int32_t* idx_out, double* mi_out, float* pred_out) {
  if (!ctx || !params || !net || net->ctx != ctx || !sur_map_ok(net, map) || n_poses <= 0 ||
      !poses || k <= 0 || k > n_poses || !idx_out || !mi_out || n_poses > (1ll << 30))
    return FSMI_E_INVAL;
  (void)hipSetDevice(ctx->device);
  int64_t npow2 = 1;
  while (npow2 < n_poses) npow2 <<= 1;
  // work: pred [n] float, key [npow2] float, idx [npow2] int, top poses [k][4] double,
  // per-beam scratch of the exact re-score [k][n_beams] double
  const size_t need = sizeof(float) * n_poses + (sizeof(float) + sizeof(int32_t)) * npow2 +
                      sizeof(double) * 4 * (size_t)k + sizeof(double) * (size_t)k * n_beams + 2048;
  if (ensure_work(ctx, need) != hipSuccess) return FSMI_E_NOMEM;
  char* w = reinterpret_cast<char*>(ctx->d_work);
  float* pred = pred_out ? pred_out : reinterpret_cast<float*>(w);
  float* key = reinterpret_cast<float*>(w + ((sizeof(float) * n_poses + 255) / 256) * 256);
  int32_t* idx = reinterpret_cast<int32_t*>(key + npow2);
  double* top = reinterpret_cast<double*>(
      reinterpret_cast<char*>(idx) + ((sizeof(int32_t) * npow2 + 255) / 256) * 256);
  fsmi_status st = fsmi_sur_forward(net, map, n_poses, poses, pred);
  if (st != FSMI_OK) return st;
  const unsigned blocks = (unsigned)((npow2 + 255) / 256);
  hipLaunchKernelGGL(k_topk_fill, dim3(blocks), dim3(256), 0, ctx->stream, n_poses, npow2, pred, key, idx);
  for (int64_t kk = 2; kk <= npow2; kk <<= 1)
    for (int64_t j = kk >> 1; j > 0; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_step, dim3(blocks), dim3(256), 0, ctx->stream, npow2, j, kk, key, idx);
  hipLaunchKernelGGL(k_gather_poses, dim3((k + 255) / 256), dim3(256), 0, ctx->stream, k, idx, poses,
                     top, idx_out);
  if (hipGetLastError() != hipSuccess) return FSMI_E_DEVICE;
  // exact re-score of the k candidates (the rank path never trusts the network alone)
  double* mb = reinterpret_cast<double*>(
      reinterpret_cast<char*>(top) + ((sizeof(double) * 4 * (size_t)k + 255) / 256) * 256);
  return fsmi_eval_poses(ctx, params, map, k, top, n_beams, beam_dir, sigma, max_range, 1.0, mi_out,
                         mb);
}

}  // extern "C"
