// 16-bit matrix-core MLS fit for gfx950 (Muelder et al., Sec. 3.3): the
// weight x feature contraction on v_mfma_f32_16x16x32_{bf16,f16} with
// float32 accumulation, followed by the float64 per-node solve.
//
// Precision design.  The normal equations amplify relative errors of the
// moments by the conditioning of the weighted basis, and a single 16-bit
// rounding of each feature (8 or 11 significant bits) is far too coarse for
// the quadratic basis.  So
//   - every feature g (moment monomial or basis x attribute) is carried as
//     an S-term expansion g = g_1 + ... + g_S of 16-bit numbers (each term
//     the rounding of what the previous terms left);
//   - the weight is carried as w_hi + w_lo (two terms) when S >= 2;
//   - the contraction issues, per feature tile, w_hi x g_s for every term
//     plus w_lo x g_s for every term but the last, all into one float32
//     accumulator (the products are exact).  What is left out,
//     w_hi g_{>S} and w_lo g_{>=S}, is about 2^-24 (bfloat16, S = 3) or
//     2^-22 (float16, S = 2) of the product for every feature alike.  With
//     w_lo x g_1 alone the product would carry w_lo (g - g_1), an error of
//     2^-16 that differs from feature to feature: the moment matrix and the
//     right-hand sides would no longer see one common weight, and the
//     normal equations amplify such inconsistent errors by their
//     conditioning;
//   - the part of the weight below w_hi + w_lo is common to all features
//     of a pair, so it only perturbs the weight function;
//   - attributes are staged in [-1, 1] (mls_stage.hip) and mapped back.
//
// Work split.  A workgroup owns a 16 x 16 node tile and one slab of
// attributes: the slab's features are the moment monomials plus
// basis x attribute products for its D_s attributes, at most 16 NTS
// columns, so the per-node accumulators fit in registers.  Every slab
// repeats the moments, which lets each slab solve its own nodes.
// Twelve waves: waves 0-7 issue the matrix instructions (each owns 2 row
// strips x NTS feature tiles of 16 x 16 float32), waves 8-11 produce.  Two
// matrix waves per SIMD let one wave build its weight operands while the
// other's MFMAs run.  Points
// stream in chunks of 64 through a three-stage pipeline, one barrier per
// chunk:
//   producers, iteration c:  load the raw chunk c + 2 (coordinates, staged
//                            attributes) from global memory into registers;
//                            turn raw chunk c + 1 (in LDS) into weight
//                            tables and 16-bit feature terms; store raw
//                            chunk c + 2 to LDS
//   MFMA waves, iteration c: build the A operands (weights) from the tables
//                            of chunk c and run its MFMAs
// so the global-memory latency of a chunk is hidden behind a whole chunk of
// matrix work.  With the Wendland weight the chunks walk the tile's list of
// cell-sorted points within reach of its nodes (mls_cells.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/mls.h"
#include "mls_internal.h"
#include "mls_solve.h"

namespace mls {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));

#ifndef MLS_LP_MMA_WAVES
#define MLS_LP_MMA_WAVES 8
#endif
constexpr int kMmaWaves = MLS_LP_MMA_WAVES;
constexpr int kProd = 256;                 // producer threads
constexpr int kThreads = kMmaWaves * 64 + kProd;
constexpr int kCols = 16;
constexpr int R = 16 / kMmaWaves;          // row strips per MFMA wave
constexpr int kRows = kMmaWaves * R;       // 16
constexpr int KT = 64;                     // points per chunk (two MFMA k-steps)
constexpr int KSF = KT + 4;                // float32 table stride (floats)
constexpr int KSH = KT + 8;                // 16-bit feature stride (elements, 144 B)
constexpr int kDsCap = 40;                 // attributes per slab at most

template <typename T> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf16x8 type; };
template <> struct Vec8<_Float16> { typedef halfx8 type; };

// Two float32 values rounded (nearest-even) to a packed pair of 16-bit
// numbers, first value in the low half: one packed conversion per pair.
template <typename T> __device__ __forceinline__ uint32_t pack2(float a, float b);
template <> __device__ __forceinline__ uint32_t pack2<__bf16>(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){a, b}, bf16x2));
}
template <> __device__ __forceinline__ uint32_t pack2<_Float16>(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){a, b}, halfx2));
}

// The same, also returning what the rounding left of each value (exact in
// float32): one term of a multi-term 16-bit expansion.
template <typename T>
__device__ __forceinline__ uint32_t pack2_rest(float a, float b, float& ra, float& rb);
template <>
__device__ __forceinline__ uint32_t pack2_rest<__bf16>(float a, float b, float& ra, float& rb) {
  const uint32_t p = pack2<__bf16>(a, b);
  ra = a - __builtin_bit_cast(float, p << 16);
  rb = b - __builtin_bit_cast(float, p & 0xFFFF0000u);
  return p;
}
template <>
__device__ __forceinline__ uint32_t pack2_rest<_Float16>(float a, float b, float& ra, float& rb) {
  const uint32_t p = pack2<_Float16>(a, b);
  const floatx2 back = __builtin_convertvector(__builtin_bit_cast(halfx2, p), floatx2);
  ra = a - back.x;
  rb = b - back.y;
  return p;
}

// Eight float32 weights as the hi + lo pair of 16-bit operands: hi is the
// rounding of w, lo the rounding of what hi leaves.
template <typename T>
__device__ __forceinline__ void split_weights(const float (&w)[8], typename Vec8<T>::type& hi,
                                              typename Vec8<T>::type& lo) {
  u32x4 h, l;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    float r0, r1;
    h[p] = pack2_rest<T>(w[2 * p], w[2 * p + 1], r0, r1);
    l[p] = pack2<T>(r0, r1);
  }
  hi = __builtin_bit_cast(typename Vec8<T>::type, h);
  lo = __builtin_bit_cast(typename Vec8<T>::type, l);
}

// Common factor applied to every weight before it is rounded to the 16-bit
// operand.  float16 has a 5-bit exponent: a Gaussian weight below 6e-5
// (r > 3.1 h) would land among its subnormals and lose most of its digits,
// so the fp16 path works with weights times 2^15 (largest 32768, still
// below the format's 65504; weights of r < 5.2 h stay normal).  bfloat16
// shares float32's exponent range and needs no factor.  The solve divides
// the weight sum by the factor before the floor test; the pivots are
// equilibrated and do not see it.
template <typename T> struct WeightGain { static constexpr float value = 1.0f; };
template <> struct WeightGain<_Float16> { static constexpr float value = 32768.0f; };

__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(halfx8 a, halfx8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

struct LPParams {
  const float* pts;       // [n][2] (cell order for the Wendland weight)
  const float* vals_t;    // [D][n] staged attributes in [-1, 1]
  const float* shift;     // [D]
  const float* scale;     // [D]
  int64_t n;
  int D, Ds, nslab;
  float inv_h;
  double inv_hd;
  double x0, y0, dx, dy;
  int W, H, tiles_x, tiles;
  double tau, floor_w;
  float cutoff2;          // points with u^2 beyond this get no features
  float* fields;
  uint8_t* deg_out;
  float* grads;           // [D][2][H][W] or null
  const uint32_t* torder;      // tile of each workgroup slot (Wendland)
  int slots;                   // workgroup slots per attribute slab (Wendland)
  const uint32_t* tile_start;  // per-tile point lists (Wendland): [tiles + 1]
  const uint32_t* tile_list;   //   cell-ordered point indices, or null
};

// A chunk: entries [k, k + kn) of the tile's point sequence (all points,
// or the tile's point list with a compactly supported weight).
struct Chunk {
  int64_t k;
  int kn;
  bool valid;
};

struct Walker {
  int64_t k, kend;
};

// Take the next chunk (invalid once the walk is over).
__device__ __forceinline__ Chunk walker_take(Walker& w) {
  Chunk c;
  c.valid = w.k < w.kend;
  c.k = w.k;
  const int64_t left = w.kend - w.k;
  c.kn = !c.valid ? 0 : (left < KT ? (int)left : KT);
  w.k += c.kn;
  return c;
}

template <int DEG, int NTS, int S, typename T>
struct LPLayout {
  static constexpr int m = DEG == 0 ? 1 : (DEG == 1 ? 3 : 6);
  static constexpr int nmom = DEG == 0 ? 1 : (DEG == 1 ? 6 : 15);
  static constexpr int kFP = NTS * 16;
  static constexpr int kDsFit = (kFP - nmom) / m > 0 ? (kFP - nmom) / m : 0;
  static constexpr int kDsMax = kDsFit < kDsCap ? kDsFit : kDsCap;
  // raw chunk: x[KT], y[KT], v[kDsMax][KT]
  static constexpr int kRawFloats = (2 + kDsMax) * KT;
  static constexpr int kRawIt = (kRawFloats + kProd - 1) / kProd;
  static constexpr int kFeatB = S * kFP * KSH * 2;            // one feature buffer
  static constexpr int kTabB = (kCols + kRows) * KSF * 4;     // one weight table
  static constexpr int kRawB = kRawFloats * 4;
  static constexpr int kFeat0 = 0;
  static constexpr int kTab0 = kFeat0 + 2 * kFeatB;
  static constexpr int kRaw0 = kTab0 + 2 * kTabB;
  static constexpr int kLoop = kRaw0 + 2 * kRawB;
  static constexpr int kEpiStride = kFP + 1;                  // floats
  static constexpr int kEpi = kMmaWaves * 16 * R * kEpiStride * 4;
  static constexpr int kBytes = kLoop > kEpi ? kLoop : kEpi;
  static_assert(kBytes <= 160 * 1024, "LDS budget");
};

// Offset of node column c0 + col (row r0 + row) from the tile anchor, in
// units of h, computed in float64 from the grid definition.
__device__ __forceinline__ double node_offset_xd(const LPParams& p, int c0, int col, float cxr) {
  return (p.x0 + (double)(c0 + col) * p.dx - (double)cxr) * p.inv_hd;
}
__device__ __forceinline__ double node_offset_yd(const LPParams& p, int r0, int row, float cyr) {
  return (p.y0 + (double)(r0 + row) * p.dy - (double)cyr) * p.inv_hd;
}

// Wendland C2 weight (1 - s)^4 (4 s + 1) for s = r / h < 1, from s^2.  The
// hardware square root (about 1 ulp) replaces the correctly rounded
// sequence, which costs eight more instructions per pair: the weight is
// carried as hi + lo bfloat16 terms, about 17 bits, and any rounding of it
// is common to every feature of the pair.
// 1 - s is clamped at 0 (a clamp bit of the subtraction), which makes the
// weight 0 from s = 1 on.
__device__ __forceinline__ float wendland_c2(float s2) {
  const float s = __builtin_amdgcn_sqrtf(s2);
  const float t = __builtin_amdgcn_fmed3f(1.0f - s, 0.0f, 1.0f);
  const float t2 = t * t;
  return t2 * t2 * (4.0f * s + 1.0f);
}

// Producer: global -> registers for one raw chunk.
// The input arrays are global memory.  Said explicitly, their loads are
// global loads also where the compiler cannot see it (parameters read from
// memory in the served batches) instead of flat loads, which also wait on
// the LDS counter.
template <typename V>
__device__ __forceinline__ const __attribute__((address_space(1))) V* global_ptr(const V* q) {
  return (const __attribute__((address_space(1))) V*)q;
}

template <int DEG, int NTS, int S, typename T>
__device__ __forceinline__ void raw_load(const LPParams& p, const Chunk& ch, int d0, int Ds,
                                         int pt, float (&r)[LPLayout<DEG, NTS, S, T>::kRawIt]) {
  using L = LPLayout<DEG, NTS, S, T>;
#pragma unroll
  for (int it = 0; it < L::kRawIt; ++it) {
    const int e = pt + it * kProd;
    float v = 0.0f;
    if (ch.valid && e < (2 + Ds) * KT) {
      const int row = e / KT, k = e - row * KT;
      if (k < ch.kn) {
        const int64_t gi =
            p.tile_list ? (int64_t)global_ptr(p.tile_list)[ch.k + k] : ch.k + k;
        if (row == 0) v = global_ptr(p.pts)[2 * gi];
        else if (row == 1) v = global_ptr(p.pts)[2 * gi + 1];
        else v = global_ptr(p.vals_t)[(int64_t)(d0 + row - 2) * p.n + gi];
      }
    }
    r[it] = v;
  }
}

template <int DEG, int NTS, int S, typename T>
__device__ __forceinline__ void raw_store(float* raw, int Ds, int pt,
                                          const float (&r)[LPLayout<DEG, NTS, S, T>::kRawIt]) {
  using L = LPLayout<DEG, NTS, S, T>;
#pragma unroll
  for (int it = 0; it < L::kRawIt; ++it) {
    const int e = pt + it * kProd;
    if (e < (2 + Ds) * KT) raw[e] = r[it];
  }
}

constexpr int kTabIt = (kCols + kRows) * KT / kProd;   // table entries per producer thread

// Node offsets (in h, from the tile anchor) of the table rows a producer
// thread fills: entry it is row (pt + it * kProd) / KT, a node column for
// rows < 16 and a node row after that.
__device__ __forceinline__ void table_offsets(const LPParams& p, int pt, int c0, int r0,
                                              float cxr, float cyr, float (&toff)[kTabIt]) {
#pragma unroll
  for (int it = 0; it < kTabIt; ++it) {
    const int row = (pt + it * kProd) / KT;
    toff[it] = row < kCols ? (float)node_offset_xd(p, c0, row, cxr)
                           : (float)node_offset_yd(p, r0, row - kCols, cyr);
  }
}

// Producer: raw chunk (LDS) -> weight tables and feature terms (LDS).
// Features: a thread owns a pair of consecutive points (pp = pt % 32) and
// one eighth of the features (group g = pt / 32): it forms the monomials of
// its two points once, then writes moment monomials j = g (mod 8) and the
// basis x attribute products of attributes d = g (mod 8), each as S packed
// 16-bit term pairs (one 32-bit LDS store per term).
template <int DEG, int NTS, int S, typename T, bool WEND>
__device__ __forceinline__ void make_chunk(const LPParams& p, const float* raw, int kn, int Ds,
                                           float* tab, T* G, int pt, const float (&toff)[kTabIt],
                                           float cxr, float cyr) {
  using L = LPLayout<DEG, NTS, S, T>;
  constexpr int m = L::m, nmom = L::nmom;
  const float* rx = raw;
  const float* ry = raw + KT;
  const float* rv = raw + 2 * KT;
  // weight tables: 32 rows (16 node columns, 16 node rows) x 64 points.
  // Gaussian: the separable factor exp(-u^2); Wendland: u^2 (combined per
  // pair when the A operand is built).  Points past the chunk: Gaussian 0,
  // Wendland a distance beyond the support.
#pragma unroll
  for (int it = 0; it < kTabIt; ++it) {
    const int e = pt + it * kProd;
    const int k = e & (KT - 1), row = e / KT;
    float v = WEND ? 4.0f : 0.0f;
    if (k < kn) {
      const float u = (row < kCols ? rx[k] - cxr : ry[k] - cyr) * p.inv_h - toff[it];
      // the fp16 weight factor rides on the column table (the weight is gx * gy)
      v = WEND ? u * u : __expf(-u * u) * (row < kCols ? WeightGain<T>::value : 1.0f);
    }
    tab[row * KSF + k] = v;
  }
  // features
  const int pp = pt & 31, g = pt >> 5;
  const int k0 = 2 * pp;
  float mo[2][nmom];
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {
    const float ux = (rx[k0 + h2] - cxr) * p.inv_h;
    const float uy = (ry[k0 + h2] - cyr) * p.inv_h;
    // points beyond the reach of every node of the tile get no features
    const float one = (ux * ux + uy * uy <= p.cutoff2) ? 1.0f : 0.0f;
    mo[h2][0] = one;
    if (nmom > 1) {
      mo[h2][1] = one * ux;
      mo[h2][2] = one * uy;
      mo[h2][3] = mo[h2][1] * ux;
      mo[h2][4] = mo[h2][1] * uy;
      mo[h2][5] = mo[h2][2] * uy;
    }
    if (nmom > 6) {
      mo[h2][6] = mo[h2][3] * ux;
      mo[h2][7] = mo[h2][3] * uy;
      mo[h2][8] = mo[h2][4] * uy;
      mo[h2][9] = mo[h2][5] * uy;
      mo[h2][10] = mo[h2][6] * ux;
      mo[h2][11] = mo[h2][6] * uy;
      mo[h2][12] = mo[h2][7] * uy;
      mo[h2][13] = mo[h2][8] * uy;
      mo[h2][14] = mo[h2][9] * uy;
    }
  }
  auto emit = [&](int j, float v0, float v1) {
    T* dst = G + (size_t)j * KSH + k0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      uint32_t pr;
      if (s + 1 < S) {
        float r0, r1;
        pr = pack2_rest<T>(v0, v1, r0, r1);
        v0 = r0;
        v1 = r1;
      } else {
        pr = pack2<T>(v0, v1);
      }
      *(uint32_t*)(dst + (size_t)s * L::kFP * KSH) = pr;
    }
  };
#pragma unroll
  for (int j = 0; j < nmom; ++j)
    if ((j & 7) == g) emit(j, mo[0][j], mo[1][j]);
  // basis term bj is monomial bj
  for (int d = g; d < Ds; d += 8) {
    const float a0 = rv[d * KT + k0], a1 = rv[d * KT + k0 + 1];
#pragma unroll
    for (int bj = 0; bj < m; ++bj) emit(nmom + bj * Ds + d, mo[0][bj] * a0, mo[1][bj] * a1);
  }
}

// One node tile and attribute slab of a fit: `block` indexes (slab, tile
// slot) as a launch's workgroup index does.  Every thread of the workgroup
// calls it with the same arguments.
template <int DEG, int NTS, int S, typename T, bool WEND, bool CELLS>
__device__ __forceinline__ void lp_tile(const LPParams& p, int block, char* lds_lp) {
  using L = LPLayout<DEG, NTS, S, T>;
  typedef typename Vec8<T>::type vec8;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool mma = wave < kMmaWaves;
  const int pt = tid - kMmaWaves * 64;   // producer thread index
  // with the cell list, p.slots workgroup slots per slab map to tiles
  // through the supertile order; empty slots return before any barrier
  const int per_slab = CELLS ? p.slots : p.tiles;
  const int slab = block / per_slab;
  const uint32_t tile_u = CELLS ? p.torder[block % per_slab] : (uint32_t)(block % per_slab);
  if (tile_u == 0xFFFFFFFFu) return;
  const int tile = (int)tile_u;
  const int c0 = (tile % p.tiles_x) * kCols;
  const int r0 = (tile / p.tiles_x) * kRows;
  const int d0 = slab * p.Ds;
  const int Ds = min(p.Ds, p.D - d0);
  // tile anchor (rounded to float32; node offsets are taken in this frame)
  const float cxr = (float)(p.x0 + (double)(c0 + kCols / 2) * p.dx);
  const float cyr = (float)(p.y0 + (double)(r0 + kRows / 2) * p.dy);

  // double buffers, selected by chunk parity b
  auto feat = [&](int b) { return (T*)(lds_lp + L::kFeat0 + b * L::kFeatB); };
  auto tab = [&](int b) { return (float*)(lds_lp + L::kTab0 + b * L::kTabB); };
  auto raw = [&](int b) { return (float*)(lds_lp + L::kRaw0 + b * L::kRawB); };

  Walker wk;
  wk.k = CELLS ? (int64_t)p.tile_start[tile] : 0;
  wk.kend = CELLS ? (int64_t)p.tile_start[tile + 1] : p.n;
  Chunk ch0 = walker_take(wk);
  Chunk ch1 = walker_take(wk);

  // feature rows past this slab's F are never written: zero them once in
  // both buffers
  {
    const int Fs = L::nmom + L::m * Ds;
    const int pad = (L::kFP - Fs) * KSH;
    for (int b = 0; b < 2; ++b)
      for (int s = 0; s < S; ++s) {
        T* z = feat(b) + ((size_t)s * L::kFP + Fs) * KSH;
        for (int e = tid; e < pad; e += kThreads) z[e] = (T)0.0f;
      }
  }
  float toff[kTabIt];
  if (!mma) table_offsets(p, pt, c0, r0, cxr, cyr, toff);

  // prologue: raw 0 and 1 to LDS, then chunk 0's tables and features
  float rr[L::kRawIt];
  if (!mma) {
    raw_load<DEG, NTS, S, T>(p, ch0, d0, Ds, pt, rr);
    raw_store<DEG, NTS, S, T>(raw(0), Ds, pt, rr);
    raw_load<DEG, NTS, S, T>(p, ch1, d0, Ds, pt, rr);
    raw_store<DEG, NTS, S, T>(raw(1), Ds, pt, rr);
  }
  __syncthreads();
  if (!mma && ch0.valid)
    make_chunk<DEG, NTS, S, T, WEND>(p, raw(0), ch0.kn, Ds, tab(0), feat(0), pt, toff, cxr, cyr);
  __syncthreads();

  floatx4 acc[R][NTS];
#pragma unroll
  for (int t = 0; t < R; ++t)
#pragma unroll
    for (int q = 0; q < NTS; ++q) acc[t][q] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int i = lane & 15;
  const int k8 = (lane >> 4) * 8;   // this lane's 8 points of a 32-point k-step
  int c = 0;
  while (ch0.valid) {
    const Chunk ch2 = walker_take(wk);
    if (mma) {
      const float* gx = tab(c & 1);
      const float* gy = tab(c & 1) + kCols * KSF;
      const T* G = feat(c & 1);
#pragma unroll
      for (int ks = 0; ks < KT; ks += 32) {
        float wx[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) wx[q] = gx[i * KSF + ks + k8 + q];
        vec8 ahi[R], alo[R];
        float smin = 4.0f;   // Wendland: the smallest u^2 among this lane's pairs
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const float* gyr = gy + (wave * R + t) * KSF + ks + k8;
          float w[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (WEND) {
              const float s2 = wx[q] + gyr[q];
              smin = fminf(smin, s2);
              w[q] = wendland_c2(s2) * WeightGain<T>::value;
            } else {
              w[q] = wx[q] * gyr[q];
            }
          }
          split_weights<T>(w, ahi[t], alo[t]);
        }
        // compact support: a k-step in which no pair of this wave's nodes
        // lies inside the support (all weights zero) adds nothing; its
        // matrix instructions are skipped
        if (WEND && !__any(smin < 1.0f)) continue;
#pragma unroll
        for (int q = 0; q < NTS; ++q) {
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const vec8 b = *(const vec8*)(G + ((size_t)s * L::kFP + q * 16 + i) * KSH + ks + k8);
#pragma unroll
            for (int t = 0; t < R; ++t) acc[t][q] = mfma16(ahi[t], b, acc[t][q]);
            if (s + 1 < S) {
#pragma unroll
              for (int t = 0; t < R; ++t) acc[t][q] = mfma16(alo[t], b, acc[t][q]);
            }
          }
        }
      }
    } else {
      raw_load<DEG, NTS, S, T>(p, ch2, d0, Ds, pt, rr);      // chunk c + 2, in flight
      if (ch1.valid)
        make_chunk<DEG, NTS, S, T, WEND>(p, raw((c + 1) & 1), ch1.kn, Ds, tab((c + 1) & 1),
                                         feat((c + 1) & 1), pt, toff, cxr, cyr);
      raw_store<DEG, NTS, S, T>(raw(c & 1), Ds, pt, rr);
    }
    __syncthreads();
    ch0 = ch1;
    ch1 = ch2;
    ++c;
  }

  // Epilogue: accumulators -> LDS [wave][node][feature] (float32) -> solve.
  float* epi = (float*)lds_lp;
  if (mma) {
    float* e = epi + wave * 16 * R * L::kEpiStride;
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int q = 0; q < NTS; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // f32 16x16 MFMA result: lane holds row 4 (lane/16) + r, column lane%16
          const int node = t * 16 + 4 * (lane >> 4) + r;
          const int feat_i = q * 16 + (lane & 15);
          e[node * L::kEpiStride + feat_i] = acc[t][q][r];
        }
  }
  __syncthreads();
  // one node per lane on the first four waves (one per SIMD): the float64
  // solve is issued by four full waves rather than eight half-empty ones
  if (tid < kRows * kCols) {
    const int w = tid / (16 * R), local = tid % (16 * R);
    const float* e = epi + (w * 16 * R + local) * L::kEpiStride;
    const int64_t plane = (int64_t)p.W * p.H;
    const int t = local / 16, col = local % 16;
    const int r = r0 + w * R + t, cc = c0 + col;
    if (r < p.H && cc < p.W) {
      const double ex = node_offset_xd(p, c0, col, cxr);
      const double ey = node_offset_yd(p, r0, w * R + t, cyr);
      const int64_t off = (int64_t)r * p.W + cc;
      uint8_t code = solve_node<DEG, float>(e, Ds, ex, ey, p.tau, p.floor_w,
                                            p.fields + (int64_t)d0 * plane + off, plane,
                                            p.shift + d0, p.scale + d0,
                                            (double)WeightGain<T>::value,
                                            p.grads ? p.grads + (int64_t)(2 * d0) * plane + off
                                                    : nullptr,
                                            p.inv_hd);
      if (p.deg_out && slab == 0) p.deg_out[off] = code;
    }
  }
}

template <int DEG, int NTS, int S, typename T, bool WEND, bool CELLS>
__global__ __launch_bounds__(kThreads) void fit_lp_kernel(LPParams p) {
  extern __shared__ __attribute__((aligned(16))) char lds_lp[];
  lp_tile<DEG, NTS, S, T, WEND, CELLS>(p, blockIdx.x, lds_lp);
}

// Persistent batch of served fits sharing one kernel shape: every
// workgroup takes (request, block) work items from a device counter until
// the list is exhausted (every workgroup reaches the end of the list, so the
// grid drains).  Before an item the request's cancel flag (host memory) is
// read; a cancelled request's items are counted but not computed, and the
// request is marked as skipped.  Items are listed request by request, so a
// workgroup meets each request in one run of items; when it moves on to the
// next request (or the list ends) it releases its output writes at device
// scope and adds the run's length to the request's count.  The workgroup
// whose addition completes a request acquires the other additions and sets
// the request's completion flag in host memory (1: every item computed, 2:
// items skipped) with a system-scope release, so the host sees each request
// finish, its outputs written, while the batch runs on.  (A release per
// item would write back the L2 after every tile, and costs about a tenth of
// the batch's time.)
struct LPBatch {
  const LPParams* __restrict__ reqs;   // [n_req]
  const uint2* items;          // [n_items] (request, block)
  const uint32_t* total;       // [n_req] items of each request
  uint32_t* head;              // next item (zero at launch)
  uint32_t* done;              // [n_req] finished items (zero at launch)
  uint32_t* skipped;           // [n_req] nonzero once an item was skipped (zero at launch)
  uint32_t* complete;          // [n_req] host: 1 or 2 when a request is done
  const uint32_t* cancel;      // [n_req] host: nonzero = skip the request
  int n_items;
};

// The tile body as a call of its own in the batch kernel, so that its
// registers are allocated apart from the item loop's.  Arguments of a call
// travel in vector registers and read as per-lane values; the parameter
// address and the block are made scalar again here, so that the parameters
// are loaded through the scalar cache as kernel arguments are, and the
// work area is named as the dynamic LDS array itself, so that its accesses
// are LDS instructions rather than flat ones.
template <int DEG, int NTS, int S, typename T>
__device__ __noinline__ void lp_tile_item(const LPParams* __restrict__ pp, int block) {
  extern __shared__ __attribute__((aligned(16))) char lds_lp[];
  // the parameter block is written before the launch and only read by the
  // kernel: in the constant address space its loads are scalar loads that
  // the compiler may repeat instead of holding their values in registers
  const uint64_t a = (uint64_t)(uintptr_t)pp;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  typedef const __attribute__((address_space(4))) LPParams* ConstParams;
  const ConstParams pc = (ConstParams)(uintptr_t)(((uint64_t)hi << 32) | lo);
  lp_tile<DEG, NTS, S, T, false, false>(*(const LPParams*)pc,
                                        __builtin_amdgcn_readfirstlane(block), lds_lp);
}

// Thread 0 takes the next item in a branch at the top of the loop; it
// counts a finished run of items in a second branch, under a condition held
// in scalar registers, and every path from there back to the top of the
// loop passes a barrier.  (With only the back edge between two thread-0
// branches the compiler threads the path of the other threads from the
// last barrier straight to the first, and the loop it builds from that runs
// their path until they leave it, which they never do: no item is taken
// without thread 0.)
template <int DEG, int NTS, int S, typename T>
__global__ __launch_bounds__(kThreads) void fit_lp_batch_kernel(LPBatch b) {
  __shared__ int sh_item, sh_skip;
  int cur_req = -1;       // request of the current run of items
  uint32_t cur_cnt = 0;   // items of the run finished here, not yet counted
  for (;;) {
    if (threadIdx.x == 0) {
      const int it = (int)atomicAdd(b.head, 1u);
      int skip = 0;
      if (it < b.n_items) {
        const uint32_t r = b.items[it].x;
        skip = __hip_atomic_load(b.cancel + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
        // released with the run's count
        if (skip) __hip_atomic_store(b.skipped + r, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      sh_item = it;
      sh_skip = skip;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(sh_item);
    const int skip = __builtin_amdgcn_readfirstlane(sh_skip);
    __syncthreads();
    const bool more = item < b.n_items;
    const uint2 w = more ? b.items[item] : make_uint2(0xFFFFFFFFu, 0u);
    const int req = __builtin_amdgcn_readfirstlane((int)w.x);   // -1 past the end
    const int block = __builtin_amdgcn_readfirstlane((int)w.y);
    if (cur_cnt > 0 && req != cur_req) {
      // the run of cur_req ends here: release its output writes, count it
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint32_t prev = atomicAdd(b.done + cur_req, cur_cnt);
        if (prev + cur_cnt == b.total[cur_req]) {
          // every item of the request is counted: acquire the other runs'
          // releases (and skip marks), then publish to the host
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          const uint32_t sk = __hip_atomic_load(b.skipped + cur_req, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(b.complete + cur_req, sk ? 2u : 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      cur_cnt = 0;
    }
    if (!more) break;
    cur_req = req;
    if (!skip) {
      // read in place (uniform, read-only): fields are loaded where used,
      // as kernel arguments are, instead of held in registers
      lp_tile_item<DEG, NTS, S, T>(b.reqs + req, block);
    }
    ++cur_cnt;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Two-pass (shape-function) form of the same fit, for the bfloat16 path with
// the Gaussian weight.  The field at node p is
//   field_d(p) = y_p^T R_t,d = sum_i w_ip (y_p^T b_t(u_i)) f_i,d,
// y_p = T'^T M_p'^{-1} e_0 the tile-frame coefficients of the node's shape
// function (mls_solve.h).  Pass 1 contracts the weights with the moment
// monomials only (one 16-column feature tile, S1 terms, split weight) and
// solves every node's ladder for y_p; pass 2 streams the points again and
// contracts the effective weights w_ip (y_p^T b_t(u_i)), formed per pair in
// float32 and split hi + lo, with the attributes (two bfloat16 terms each).
// The contraction width falls from n_mom + m D to n_mom + D (399 -> 79 for
// the quadratic basis with 64 attributes); the solve runs once per node and
// attribute slab instead of per feature.  The error stays the float32
// accumulation of the moments in pass 1: the effective weights and the
// attribute terms add about 2^-16 relative per pair, which is not amplified
// by the conditioning (a numpy model of both forms gives the same error).
// ---------------------------------------------------------------------------

constexpr int kShapeDsCap = 64;    // attributes per workgroup slab
constexpr int kShapeS2 = 2;        // bfloat16 terms per attribute value

template <int DEG, int NTV, int S1>
struct ShapeLayout {
  static constexpr int m = DEG == 1 ? 3 : 6;
  static constexpr int nmom = DEG == 1 ? 6 : 15;
  static constexpr int kRows1 = S1 * 16;                 // pass 1 feature rows
  static constexpr int kRows2 = kShapeS2 * NTV * 16;     // pass 2 feature rows
  static constexpr int kFeatRows = kRows1 > kRows2 ? kRows1 : kRows2;
  static constexpr int kDs = NTV * 16;
  static constexpr int kRawFloats = (2 + kDs) * KT;
  static constexpr int kRawIt = (kRawFloats + kProd - 1) / kProd;
  static constexpr int kFeatB = kFeatRows * KSH * 2;
  static constexpr int kTabB = (kCols + kRows) * KSF * 4;
  static constexpr int kBasB = 3 * KSF * 4;              // 1, u_x, u_y per point
  static constexpr int kRawB = kRawFloats * 4;
  static constexpr int kFeat0 = 0;
  static constexpr int kTab0 = kFeat0 + 2 * kFeatB;
  static constexpr int kBas0 = kTab0 + 2 * kTabB;
  static constexpr int kRaw0 = kBas0 + 2 * kBasB;
  static constexpr int kLoop = kRaw0 + 2 * kRawB;
  static constexpr int kEpiStride = 16 + 1;
  static constexpr int kEpi = kMmaWaves * 16 * R * kEpiStride * 4;
  static constexpr int kMain = kLoop > kEpi ? kLoop : kEpi;
  // per node: the shape coefficients y (float32) and the degree code
  static constexpr int kY0 = kMain;
  static constexpr int kCode0 = kY0 + kRows * kCols * m * 4;
  static constexpr int kBytes = kCode0 + kRows * kCols;
  static_assert(kBytes <= 160 * 1024, "LDS budget");
};

// Producer: global -> registers for one raw chunk of `nv` attributes.
template <int RAWIT>
__device__ __forceinline__ void shape_raw_load(const LPParams& p, const Chunk& ch, int d0, int nv,
                                               int pt, float (&r)[RAWIT]) {
#pragma unroll
  for (int it = 0; it < RAWIT; ++it) {
    const int e = pt + it * kProd;
    float v = 0.0f;
    if (ch.valid && e < (2 + nv) * KT) {
      const int row = e / KT, k = e - row * KT;
      if (k < ch.kn) {
        const int64_t gi = ch.k + k;
        if (row == 0) v = p.pts[2 * gi];
        else if (row == 1) v = p.pts[2 * gi + 1];
        else v = p.vals_t[(int64_t)(d0 + row - 2) * p.n + gi];
      }
    }
    r[it] = v;
  }
}

template <int RAWIT>
__device__ __forceinline__ void shape_raw_store(float* raw, int nv, int pt,
                                                const float (&r)[RAWIT]) {
#pragma unroll
  for (int it = 0; it < RAWIT; ++it) {
    const int e = pt + it * kProd;
    if (e < (2 + nv) * KT) raw[e] = r[it];
  }
}

// Producer: the separable Gaussian tables of a chunk (32 rows: 16 node
// columns, then 16 node rows, x 64 points; zero past the chunk).
__device__ __forceinline__ void gauss_tables(const LPParams& p, const float* raw, int kn,
                                             float* tab, int pt, const float (&toff)[kTabIt],
                                             float cxr, float cyr) {
#pragma unroll
  for (int it = 0; it < kTabIt; ++it) {
    const int e = pt + it * kProd;
    const int k = e & (KT - 1), row = e / KT;
    float v = 0.0f;
    if (k < kn) {
      const float u = (row < kCols ? raw[k] - cxr : raw[KT + k] - cyr) * p.inv_h - toff[it];
      v = __expf(-u * u);
    }
    tab[row * KSF + k] = v;
  }
}

// Split two float32 values into `S` bfloat16 terms each (each term the
// rounding of what the earlier ones left), written as pairs at rows
// dst + s * stride.
template <int S>
__device__ __forceinline__ void emit_terms(__bf16* dst, size_t stride, float v0, float v1) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    uint32_t pr;
    if (s + 1 < S) {
      float r0, r1;
      pr = pack2_rest<__bf16>(v0, v1, r0, r1);
      v0 = r0;
      v1 = r1;
    } else {
      pr = pack2<__bf16>(v0, v1);
    }
    *(uint32_t*)(dst + (size_t)s * stride) = pr;
  }
}

// Monomials u_x^a u_y^b (a + b <= 2 DEG) of a point in the tile frame, in
// mono_index order; zero for points beyond the reach of every node.
template <int DEG>
__device__ __forceinline__ void point_monomials(const LPParams& p, float x, float y, float cxr,
                                                float cyr, float (&mo)[DEG == 1 ? 6 : 15]) {
  const float ux = (x - cxr) * p.inv_h;
  const float uy = (y - cyr) * p.inv_h;
  const float one = (ux * ux + uy * uy <= p.cutoff2) ? 1.0f : 0.0f;
  mo[0] = one;
  mo[1] = one * ux;
  mo[2] = one * uy;
  mo[3] = mo[1] * ux;
  mo[4] = mo[1] * uy;
  mo[5] = mo[2] * uy;
  if (DEG == 2) {
    mo[6] = mo[3] * ux;
    mo[7] = mo[3] * uy;
    mo[8] = mo[4] * uy;
    mo[9] = mo[5] * uy;
    mo[10] = mo[6] * ux;
    mo[11] = mo[6] * uy;
    mo[12] = mo[7] * uy;
    mo[13] = mo[8] * uy;
    mo[14] = mo[9] * uy;
  }
}

// Producer, pass 1: tables and the moment monomials (S1 terms, rows
// s * 16 + j).  Pass 2: tables, the basis values u_x, u_y of the chunk's
// points (float32, rows 1-2 of `bas`; zero past the reach), and the
// attribute terms (rows s * kDs + d), zero past the reach: a point beyond
// every node's reach then adds nothing whatever its effective weight, so
// the matrix lanes need no reach mask of their own.
// A thread owns two consecutive points and one eighth of the rows.
template <int DEG, int NTV, int S1, bool PASS2>
__device__ __forceinline__ void shape_chunk(const LPParams& p, const float* raw, int kn, int nv,
                                            float* tab, float* bas, __bf16* G, int pt,
                                            const float (&toff)[kTabIt], float cxr,
                                            float cyr) {
  using L = ShapeLayout<DEG, NTV, S1>;
  gauss_tables(p, raw, kn, tab, pt, toff, cxr, cyr);
  const int pp = pt & 31, g = pt >> 5;
  const int k0 = 2 * pp;
  float mo0[L::nmom], mo1[L::nmom];
  point_monomials<DEG>(p, raw[k0], raw[KT + k0], cxr, cyr, mo0);
  point_monomials<DEG>(p, raw[k0 + 1], raw[KT + k0 + 1], cxr, cyr, mo1);
  if (!PASS2) {
#pragma unroll
    for (int j = 0; j < L::nmom; ++j)
      if ((j & 7) == g) emit_terms<S1>(G + (size_t)j * KSH + k0, (size_t)16 * KSH, mo0[j], mo1[j]);
    return;
  }
#pragma unroll
  for (int j = 1; j < 3; ++j)   // u_x, u_y (the matrix waves form the rest)
    if ((j & 7) == g) {
      bas[j * KSF + k0] = mo0[j];
      bas[j * KSF + k0 + 1] = mo1[j];
    }
  const float* rv = raw + 2 * KT;
  for (int d = g; d < nv; d += 8)
    emit_terms<kShapeS2>(G + (size_t)d * KSH + k0, (size_t)L::kDs * KSH,
                         mo0[0] * rv[d * KT + k0], mo1[0] * rv[d * KT + k0 + 1]);
}

template <int DEG, int NTV, int S1>
__global__ __launch_bounds__(kThreads) void fit_shape_kernel(LPParams p) {
  using L = ShapeLayout<DEG, NTV, S1>;
  constexpr int m = L::m;
  extern __shared__ __attribute__((aligned(16))) char lds_sh[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool mma = wave < kMmaWaves;
  const int pt = tid - kMmaWaves * 64;
  const int slab = blockIdx.x / p.tiles;
  const int tile = (int)(blockIdx.x % p.tiles);
  const int c0 = (tile % p.tiles_x) * kCols;
  const int r0 = (tile / p.tiles_x) * kRows;
  const int d0 = slab * p.Ds;
  const int nv = min(p.Ds, p.D - d0);
  const float cxr = (float)(p.x0 + (double)(c0 + kCols / 2) * p.dx);
  const float cyr = (float)(p.y0 + (double)(r0 + kRows / 2) * p.dy);

  auto feat = [&](int b) { return (__bf16*)(lds_sh + L::kFeat0 + b * L::kFeatB); };
  auto tab = [&](int b) { return (float*)(lds_sh + L::kTab0 + b * L::kTabB); };
  auto bas = [&](int b) { return (float*)(lds_sh + L::kBas0 + b * L::kBasB); };
  auto raw = [&](int b) { return (float*)(lds_sh + L::kRaw0 + b * L::kRawB); };
  float* ybuf = (float*)(lds_sh + L::kY0);
  uint8_t* codes = (uint8_t*)(lds_sh + L::kCode0);

  float toff[kTabIt];
  if (!mma) table_offsets(p, pt, c0, r0, cxr, cyr, toff);
  const int i = lane & 15;
  const int k8 = (lane >> 4) * 8;
  const int64_t plane = (int64_t)p.W * p.H;

  // ---- pass 1: moments, then the ladder and the shape coefficients ----
  {
    // feature rows past the moments are never written: zero them once
    for (int b = 0; b < 2; ++b)
      for (int s = 0; s < S1; ++s) {
        __bf16* z = feat(b) + ((size_t)s * 16 + L::nmom) * KSH;
        for (int e = tid; e < (16 - L::nmom) * KSH; e += kThreads) z[e] = (__bf16)0.0f;
      }
    Walker wk{0, p.n};
    Chunk ch0 = walker_take(wk);
    Chunk ch1 = walker_take(wk);
    float rr[L::kRawIt];
    if (!mma) {
      shape_raw_load<L::kRawIt>(p, ch0, d0, 0, pt, rr);
      shape_raw_store<L::kRawIt>(raw(0), 0, pt, rr);
      shape_raw_load<L::kRawIt>(p, ch1, d0, 0, pt, rr);
      shape_raw_store<L::kRawIt>(raw(1), 0, pt, rr);
    }
    __syncthreads();
    if (!mma && ch0.valid)
      shape_chunk<DEG, NTV, S1, false>(p, raw(0), ch0.kn, 0, tab(0), bas(0), feat(0), pt, toff,
                                       cxr, cyr);
    __syncthreads();
    floatx4 acc[R];
#pragma unroll
    for (int t = 0; t < R; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    int c = 0;
    while (ch0.valid) {
      const Chunk ch2 = walker_take(wk);
      if (mma) {
        const float* gx = tab(c & 1);
        const float* gy = tab(c & 1) + kCols * KSF;
        const __bf16* G = feat(c & 1);
#pragma unroll
        for (int ks = 0; ks < KT; ks += 32) {
          float wx[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) wx[q] = gx[i * KSF + ks + k8 + q];
          bf16x8 ahi[R], alo[R];
#pragma unroll
          for (int t = 0; t < R; ++t) {
            const float* gyr = gy + (wave * R + t) * KSF + ks + k8;
            float w[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) w[q] = wx[q] * gyr[q];
            split_weights<__bf16>(w, ahi[t], alo[t]);
          }
#pragma unroll
          for (int s = 0; s < S1; ++s) {
            const bf16x8 b = *(const bf16x8*)(G + ((size_t)s * 16 + i) * KSH + ks + k8);
#pragma unroll
            for (int t = 0; t < R; ++t) acc[t] = mfma16(ahi[t], b, acc[t]);
            if (s + 1 < S1) {
#pragma unroll
              for (int t = 0; t < R; ++t) acc[t] = mfma16(alo[t], b, acc[t]);
            }
          }
        }
      } else {
        shape_raw_load<L::kRawIt>(p, ch2, d0, 0, pt, rr);
        if (ch1.valid)
          shape_chunk<DEG, NTV, S1, false>(p, raw((c + 1) & 1), ch1.kn, 0, tab((c + 1) & 1),
                                           bas((c + 1) & 1), feat((c + 1) & 1), pt, toff, cxr,
                                           cyr);
        shape_raw_store<L::kRawIt>(raw(c & 1), 0, pt, rr);
      }
      __syncthreads();
      ch0 = ch1;
      ch1 = ch2;
      ++c;
    }
    // moments -> LDS [wave][node][monomial], then one node per lane: the
    // ladder, the degree code and y (float32)
    float* epi = (float*)lds_sh;
    if (mma) {
      float* e = epi + wave * 16 * R * L::kEpiStride;
#pragma unroll
      for (int t = 0; t < R; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          e[(t * 16 + 4 * (lane >> 4) + r) * L::kEpiStride + (lane & 15)] = acc[t][r];
    }
    __syncthreads();
    // one node per lane on the first four waves (one per SIMD)
    if (tid < kRows * kCols) {
      const int w = tid / (16 * R), local = tid % (16 * R);
      const float* e = epi + (w * 16 * R + local) * L::kEpiStride;
      const int t = local / 16, col = local % 16;
      const int row = w * R + t;
      const double ex = node_offset_xd(p, c0, col, cxr);
      const double ey = node_offset_yd(p, r0, row, cyr);
      Ladder<DEG> lad;
      const int code = ladder_solve<DEG>(e, ex, ey, p.tau, p.floor_w, 1.0, lad);
      float* yv = ybuf + (row * kCols + col) * m;
#pragma unroll
      for (int j = 0; j < m; ++j) yv[j] = code == 255 ? 0.0f : (float)lad.y[j];
      codes[row * kCols + col] = (uint8_t)code;
      const int rr2 = r0 + row, cc = c0 + col;
      if (p.deg_out && slab == 0 && rr2 < p.H && cc < p.W)
        p.deg_out[(int64_t)rr2 * p.W + cc] = (uint8_t)code;
    }
    __syncthreads();
  }

  // ---- pass 2: effective weights x attribute terms ----
  {
    // attribute rows past this slab's values are never written: zero them
    for (int b = 0; b < 2; ++b)
      for (int s = 0; s < kShapeS2; ++s) {
        __bf16* z = feat(b) + ((size_t)s * L::kDs + nv) * KSH;
        for (int e = tid; e < (L::kDs - nv) * KSH; e += kThreads) z[e] = (__bf16)0.0f;
      }
    // the shape coefficients of this lane's nodes (column i of its strips)
    float yv[R][m];
    if (mma) {
#pragma unroll
      for (int t = 0; t < R; ++t)
#pragma unroll
        for (int j = 0; j < m; ++j) yv[t][j] = ybuf[((wave * R + t) * kCols + i) * m + j];
    }
    Walker wk{0, p.n};
    Chunk ch0 = walker_take(wk);
    Chunk ch1 = walker_take(wk);
    float rr[L::kRawIt];
    if (!mma) {
      shape_raw_load<L::kRawIt>(p, ch0, d0, nv, pt, rr);
      shape_raw_store<L::kRawIt>(raw(0), nv, pt, rr);
      shape_raw_load<L::kRawIt>(p, ch1, d0, nv, pt, rr);
      shape_raw_store<L::kRawIt>(raw(1), nv, pt, rr);
    }
    __syncthreads();
    if (!mma && ch0.valid)
      shape_chunk<DEG, NTV, S1, true>(p, raw(0), ch0.kn, nv, tab(0), bas(0), feat(0), pt, toff,
                                      cxr, cyr);
    __syncthreads();
    floatx4 acc[R][NTV];
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int q = 0; q < NTV; ++q) acc[t][q] = floatx4{0.f, 0.f, 0.f, 0.f};
    int c = 0;
    while (ch0.valid) {
      const Chunk ch2 = walker_take(wk);
      if (mma) {
        const float* gx = tab(c & 1);
        const float* gy = tab(c & 1) + kCols * KSF;
        const float* bs = bas(c & 1);
        const __bf16* G = feat(c & 1);
#pragma unroll
        for (int ks = 0; ks < KT; ks += 32) {
          bf16x8 ahi[R], alo[R];
          u32x4 hv[R], lv[R];
          // two points at a time: their basis values and column factors,
          // then the effective weight of each of the lane's nodes, split
          // hi + lo with one packed conversion per pair
#pragma unroll
          for (int q = 0; q < 8; q += 2) {
            float w[R][2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const int k = ks + k8 + q + e;
              // b = (1, u_x, u_y[, u_x^2, u_x u_y, u_y^2]): the quadratic
              // terms follow from the linear ones (Horner), so a point
              // needs two values, not five (past the reach its attribute
              // terms are zero)
              const float b1 = bs[KSF + k], b2 = bs[2 * KSF + k];
              const float wxq = gx[i * KSF + k];
#pragma unroll
              for (int t = 0; t < R; ++t) {
                float sh;
                if (DEG == 1) {
                  sh = fmaf(yv[t][2], b2, fmaf(yv[t][1], b1, yv[t][0]));
                } else {
                  const float s1 = fmaf(yv[t][3], b1, fmaf(yv[t][4], b2, yv[t][1]));
                  const float s2 = fmaf(yv[t][5], b2, yv[t][2]);
                  sh = fmaf(b1, s1, fmaf(b2, s2, yv[t][0]));
                }
                w[t][e] = (wxq * gy[(wave * R + t) * KSF + k]) * sh;
              }
            }
#pragma unroll
            for (int t = 0; t < R; ++t) {
              float r0, r1;
              hv[t][q / 2] = pack2_rest<__bf16>(w[t][0], w[t][1], r0, r1);
              lv[t][q / 2] = pack2<__bf16>(r0, r1);
            }
          }
#pragma unroll
          for (int t = 0; t < R; ++t) {
            ahi[t] = __builtin_bit_cast(bf16x8, hv[t]);
            alo[t] = __builtin_bit_cast(bf16x8, lv[t]);
          }
#pragma unroll
          for (int q = 0; q < NTV; ++q) {
            const bf16x8 b1 = *(const bf16x8*)(G + ((size_t)q * 16 + i) * KSH + ks + k8);
            const bf16x8 b2 =
                *(const bf16x8*)(G + ((size_t)L::kDs + q * 16 + i) * KSH + ks + k8);
#pragma unroll
            for (int t = 0; t < R; ++t) {
              acc[t][q] = mfma16(ahi[t], b1, acc[t][q]);
              acc[t][q] = mfma16(alo[t], b1, acc[t][q]);
              acc[t][q] = mfma16(ahi[t], b2, acc[t][q]);
            }
          }
        }
      } else {
        shape_raw_load<L::kRawIt>(p, ch2, d0, nv, pt, rr);
        if (ch1.valid)
          shape_chunk<DEG, NTV, S1, true>(p, raw((c + 1) & 1), ch1.kn, nv, tab((c + 1) & 1),
                                          bas((c + 1) & 1), feat((c + 1) & 1), pt, toff, cxr,
                                          cyr);
        shape_raw_store<L::kRawIt>(raw(c & 1), nv, pt, rr);
      }
      __syncthreads();
      ch0 = ch1;
      ch1 = ch2;
      ++c;
    }
    // fields: the accumulators are the normalised values; lane holds node
    // columns 4 (lane / 16) + r of strip t for attribute q * 16 + lane % 16
    if (mma) {
#pragma unroll
      for (int q = 0; q < NTV; ++q) {
        const int dd = q * 16 + (lane & 15);
        if (dd >= nv) continue;
        const double sh = (double)p.shift[d0 + dd], sc = (double)p.scale[d0 + dd];
        float* fd = p.fields + (int64_t)(d0 + dd) * plane;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int row = wave * R + t, rg = r0 + row;
          if (rg >= p.H) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = 4 * (lane >> 4) + r, cg = c0 + col;
            if (cg >= p.W) continue;
            const bool und = codes[row * kCols + col] == 255;
            fd[(int64_t)rg * p.W + cg] =
                und ? __builtin_nanf("") : (float)(sh + sc * (double)acc[t][q][r]);
          }
        }
      }
    }
  }
}

template <int DEG, int NTV, int S1>
hipError_t launch_shape_impl(const LPParams& p, hipStream_t s) {
  using L = ShapeLayout<DEG, NTV, S1>;
  const size_t lds = (size_t)L::kBytes;
  const void* fn = (const void*)fit_shape_kernel<DEG, NTV, S1>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t blocks = (int64_t)p.tiles * p.nslab;
  hipLaunchKernelGGL((fit_shape_kernel<DEG, NTV, S1>), dim3((unsigned)blocks), dim3(kThreads), lds,
                     s, p);
  return hipGetLastError();
}

template <int DEG, int S1>
hipError_t launch_shape_ntv(const LPParams& p, int ntv, hipStream_t s) {
  switch (ntv) {
    case 1: return launch_shape_impl<DEG, 1, S1>(p, s);
    case 2: return launch_shape_impl<DEG, 2, S1>(p, s);
    case 3: return launch_shape_impl<DEG, 3, S1>(p, s);
    default: return launch_shape_impl<DEG, 4, S1>(p, s);
  }
}

template <int S1>
hipError_t launch_shape_deg(const LPParams& p, int deg, int ntv, hipStream_t s) {
  return deg == 1 ? launch_shape_ntv<1, S1>(p, ntv, s) : launch_shape_ntv<2, S1>(p, ntv, s);
}

template <int DEG, int NTS, int S, typename T, bool WEND>
hipError_t launch_lp_impl(LPParams p, hipStream_t s) {
  using L = LPLayout<DEG, NTS, S, T>;
  const size_t lds = (size_t)L::kBytes;
  // Wendland weights always walk the cell list; the Gaussian runs dense
  const void* fn = WEND ? (const void*)fit_lp_kernel<DEG, NTS, S, T, true, true>
                        : (const void*)fit_lp_kernel<DEG, NTS, S, T, false, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t blocks = (int64_t)(WEND ? p.slots : p.tiles) * p.nslab;
  if (WEND)
    hipLaunchKernelGGL((fit_lp_kernel<DEG, NTS, S, T, true, true>), dim3((unsigned)blocks),
                       dim3(kThreads), lds, s, p);
  else
    hipLaunchKernelGGL((fit_lp_kernel<DEG, NTS, S, T, false, false>), dim3((unsigned)blocks),
                       dim3(kThreads), lds, s, p);
  return hipGetLastError();
}

template <int DEG, int S, typename T, bool WEND>
hipError_t launch_lp_nts(const LPParams& p, int nts, hipStream_t s) {
  switch (nts) {
    case 1: return launch_lp_impl<DEG, 1, S, T, WEND>(p, s);
    case 2: return launch_lp_impl<DEG, 2, S, T, WEND>(p, s);
    case 3: return launch_lp_impl<DEG, 3, S, T, WEND>(p, s);
    case 4: return launch_lp_impl<DEG, 4, S, T, WEND>(p, s);
    case 5: return launch_lp_impl<DEG, 5, S, T, WEND>(p, s);
    case 6: return launch_lp_impl<DEG, 6, S, T, WEND>(p, s);
    case 7: return launch_lp_impl<DEG, 7, S, T, WEND>(p, s);
    default: return launch_lp_impl<DEG, 8, S, T, WEND>(p, s);
  }
}

template <int S, typename T, bool WEND>
hipError_t launch_lp_deg(const LPParams& p, int deg, int nts, hipStream_t s) {
  switch (deg) {
    case 0: return launch_lp_nts<0, S, T, WEND>(p, nts, s);
    case 1: return launch_lp_nts<1, S, T, WEND>(p, nts, s);
    default: return launch_lp_nts<2, S, T, WEND>(p, nts, s);
  }
}

template <typename T, bool WEND>
hipError_t launch_lp_terms(const LPParams& p, int deg, int nts, int terms, hipStream_t s) {
  switch (terms) {
    case 1: return launch_lp_deg<1, T, WEND>(p, deg, nts, s);
    case 2: return launch_lp_deg<2, T, WEND>(p, deg, nts, s);
    default: return launch_lp_deg<3, T, WEND>(p, deg, nts, s);
  }
}

}  // namespace

// Slab plan: feature tiles per slab (1..8) and attributes per slab (at most
// kDsCap) that cover D with the fewest padded columns in total.
static_assert((8 * 16 - 1) / 1 >= MLS_LP_MAX_SLAB_CONSTANT && kDsCap == MLS_LP_MAX_SLAB_CONSTANT,
              "constant-basis slab limit");
static_assert((8 * 16 - 6) / 3 >= MLS_LP_MAX_SLAB_LINEAR && kDsCap == MLS_LP_MAX_SLAB_LINEAR,
              "linear-basis slab limit");
static_assert((8 * 16 - 15) / 6 == MLS_LP_MAX_SLAB_QUADRATIC, "quadratic-basis slab limit");

int lp_max_slab(int degree) {
  const int m = basis_terms(degree), nmom = moment_terms(degree);
  const int ds = (8 * 16 - nmom) / m;
  return ds < kDsCap ? ds : kDsCap;
}

void lp_slab_plan(int degree, int D, int forced_ds, int* nts_out, int* ds_out, int* nslab_out) {
  const int m = basis_terms(degree), nmom = moment_terms(degree);
  if (forced_ds > 0) {
    const int ds = forced_ds < D ? forced_ds : D;
    int nts = 1;
    while (nts * 16 < nmom + m * ds) ++nts;
    *nts_out = nts;
    *ds_out = ds;
    *nslab_out = (D + ds - 1) / ds;
    return;
  }
  int best_cost = 1 << 30, best_nts = 8, best_ds = 1, best_ns = D;
  for (int nts = 1; nts <= 8; ++nts) {
    int ds = (nts * 16 - nmom) / m;
    if (ds > kDsCap) ds = kDsCap;
    if (ds < 1) continue;
    const int dsu = ds < D ? ds : D;
    const int ns = (D + dsu - 1) / dsu;
    const int cost = ns * nts;
    if (cost < best_cost || (cost == best_cost && nts > best_nts)) {
      best_cost = cost;
      best_nts = nts;
      best_ds = dsu;
      best_ns = ns;
    }
  }
  // the smallest tile count that still holds best_ds attributes
  int nts = 1;
  while (nts * 16 < nmom + m * best_ds) ++nts;
  *nts_out = nts;
  *ds_out = best_ds;
  *nslab_out = best_ns;
}

// ---- served batches ----

bool lp_batch_class(const FitArgs& a, bool fp16, int terms, LPBatchClass* cls) {
  if (a.wkind != 0 || a.grads || a.rigid) return false;
  // batch kernels exist for each format's default term count
  if (terms != (fp16 ? 2 : 3)) return false;
  if (lp_use_shape_form(a.degree, a.D, fp16, a.wkind, false, terms, 0, a.lp_form)) return false;
  int nts, ds, nslab;
  lp_slab_plan(a.degree, a.D, a.lp_slab, &nts, &ds, &nslab);
  cls->deg = a.degree;
  cls->nts = nts;
  cls->terms = terms;
  cls->fp16 = fp16;
  const int64_t tiles = (int64_t)((a.W + kCols - 1) / kCols) * ((a.H + kRows - 1) / kRows);
  cls->blocks = tiles * nslab;
  return true;
}

size_t lp_params_bytes() { return sizeof(LPParams); }

// Parameters of a one-pass fit (launch_fit_lp and the served batches).
static LPParams dense_lp_params(const FitArgs& a, const float* vals_t, const float* shift,
                                const float* scale) {
  int nts, ds, nslab;
  lp_slab_plan(a.degree, a.D, a.lp_slab, &nts, &ds, &nslab);
  LPParams p{};
  p.pts = a.pts;
  p.vals_t = vals_t;
  p.shift = shift;
  p.scale = scale;
  p.n = a.n;
  p.D = a.D;
  p.Ds = ds;
  p.nslab = nslab;
  p.inv_hd = 1.0 / a.h;
  p.inv_h = (float)p.inv_hd;
  p.x0 = a.x0; p.y0 = a.y0; p.dx = a.dx; p.dy = a.dy;
  p.W = a.W; p.H = a.H;
  p.tiles_x = (a.W + kCols - 1) / kCols;
  p.tiles = p.tiles_x * ((a.H + kRows - 1) / kRows);
  p.tau = a.tau;
  p.floor_w = a.floor_w;
  // weight below exp(-64) ~ 1.6e-28 at every node of the tile: the tile
  // spans at most half its diagonal from the anchor
  const double sxd = a.dx / a.h, syd = a.dy / a.h;
  const double half = 0.5 * sqrt((double)(kCols * kCols) * sxd * sxd +
                                 (double)(kRows * kRows) * syd * syd);
  const double reach = 8.0 + half;
  p.cutoff2 = (float)(reach * reach);
  p.fields = a.fields;
  p.deg_out = a.deg_out;
  p.grads = nullptr;
  p.torder = nullptr;
  p.tile_start = nullptr;
  p.tile_list = nullptr;
  return p;
}

void lp_params_write(const FitArgs& a, const float* vals_t, const float* shift,
                     const float* scale, void* out) {
  const LPParams p = dense_lp_params(a, vals_t, shift, scale);
  memcpy(out, &p, sizeof(p));
}

// One workgroup per resident slot of the device (compute units x the
// kernel's occupancy), at most one per item, at most max_grid if nonzero.
template <int DEG, int NTS, int S, typename T>
hipError_t launch_batch_impl(const LPBatch& b, int max_grid, hipStream_t s) {
  using L = LPLayout<DEG, NTS, S, T>;
  const size_t lds = (size_t)L::kBytes;
  const void* fn = (const void*)fit_lp_batch_kernel<DEG, NTS, S, T>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds)) !=
      hipSuccess)
    return e;
  int64_t grid = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  if (grid > b.n_items) grid = b.n_items;
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  if (grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fit_lp_batch_kernel<DEG, NTS, S, T>), dim3((unsigned)grid), dim3(kThreads),
                     lds, s, b);
  return hipGetLastError();
}

template <int DEG, int S, typename T>
hipError_t launch_batch_nts(const LPBatch& b, int nts, int grid, hipStream_t s) {
  switch (nts) {
    case 1: return launch_batch_impl<DEG, 1, S, T>(b, grid, s);
    case 2: return launch_batch_impl<DEG, 2, S, T>(b, grid, s);
    case 3: return launch_batch_impl<DEG, 3, S, T>(b, grid, s);
    case 4: return launch_batch_impl<DEG, 4, S, T>(b, grid, s);
    case 5: return launch_batch_impl<DEG, 5, S, T>(b, grid, s);
    case 6: return launch_batch_impl<DEG, 6, S, T>(b, grid, s);
    case 7: return launch_batch_impl<DEG, 7, S, T>(b, grid, s);
    default: return launch_batch_impl<DEG, 8, S, T>(b, grid, s);
  }
}

template <int S, typename T>
hipError_t launch_batch_deg(const LPBatch& b, int deg, int nts, int grid, hipStream_t s) {
  switch (deg) {
    case 0: return launch_batch_nts<0, S, T>(b, nts, grid, s);
    case 1: return launch_batch_nts<1, S, T>(b, nts, grid, s);
    default: return launch_batch_nts<2, S, T>(b, nts, grid, s);
  }
}


hipError_t launch_fit_lp_batch(const LPBatchClass& c, const void* d_params, const uint32_t* d_items,
                               int n_items, const uint32_t* d_total, uint32_t* d_head,
                               uint32_t* d_done, uint32_t* d_skipped, uint32_t* h_complete,
                               const uint32_t* h_cancel, int grid, hipStream_t s) {
  LPBatch b;
  b.reqs = (const LPParams*)d_params;
  b.items = (const uint2*)d_items;
  b.total = d_total;
  b.head = d_head;
  b.done = d_done;
  b.skipped = d_skipped;
  b.complete = h_complete;
  b.cancel = h_cancel;
  b.n_items = n_items;
  if (c.terms != (c.fp16 ? 2 : 3)) return hipErrorInvalidValue;
  return c.fp16 ? launch_batch_deg<2, _Float16>(b, c.deg, c.nts, grid, s)
                : launch_batch_deg<3, __bf16>(b, c.deg, c.nts, grid, s);
}

// Largest node offset across a tile, in units of h.
double lp_tile_extent(double dx, double dy, double h) {
  const double ex = (double)(kCols - 1) * fabs(dx / h), ey = (double)(kRows - 1) * fabs(dy / h);
  return ex > ey ? ex : ey;
}

bool lp_use_shape_form(int degree, int D, bool fp16, int wkind, bool grads, int terms,
                       int forced_ds, int form) {
  if (fp16 || wkind != 0 || grads || degree < 1) return false;
  if (form == 1) return false;
  if (form == 2) return true;
  // the library's choice: the two-pass form once the one-pass form would
  // issue at least twice its matrix instructions
  int nts, ds, nslab;
  lp_slab_plan(degree, D, forced_ds, &nts, &ds, &nslab);
  const int one = nslab * nts * (2 * terms - 1);
  const int nslab2 = (D + kShapeDsCap - 1) / kShapeDsCap;
  const int per2 = (D + nslab2 - 1) / nslab2;
  const int two = nslab2 * ((2 * terms - 1) + 3 * ((per2 + 15) / 16));
  return one >= 2 * two;
}

hipError_t launch_fit_lp(const FitArgs& a, const float* vals_t, const float* shift,
                         const float* scale, bool fp16, int terms, const LPCells* cells,
                         hipStream_t stream) {
  // the form depends on the request, not on the slab width (a tuning knob
  // that must not change a result bit)
  if (lp_use_shape_form(a.degree, a.D, fp16, a.wkind, a.grads != nullptr, terms, 0,
                        a.lp_form)) {
    LPParams p = dense_lp_params(a, vals_t, shift, scale);
    p.nslab = (a.D + kShapeDsCap - 1) / kShapeDsCap;
    p.Ds = (a.D + p.nslab - 1) / p.nslab;
    const int ntv = (p.Ds + 15) / 16;
    switch (terms) {
      case 1: return launch_shape_deg<1>(p, a.degree, ntv, stream);
      case 2: return launch_shape_deg<2>(p, a.degree, ntv, stream);
      default: return launch_shape_deg<3>(p, a.degree, ntv, stream);
    }
  }
  // the same parameters a served batch passes for the request, so that a
  // request computes the same bits alone and in a batch
  int nts, ds, nslab;
  lp_slab_plan(a.degree, a.D, a.lp_slab, &nts, &ds, &nslab);
  LPParams p = dense_lp_params(a, vals_t, shift, scale);
  p.grads = a.grads;
  const bool wend = a.wkind == 1;
  if (wend) {
    if (!cells) return hipErrorInvalidValue;
    p.pts = cells->pts_s;
    p.vals_t = cells->vals_ts;
    p.torder = cells->torder;
    p.slots = (int)tile_order_slots(p.tiles_x, p.tiles / p.tiles_x);
    p.tile_start = cells->tile_start;
    p.tile_list = cells->tile_list;
    return fp16 ? launch_lp_terms<_Float16, true>(p, a.degree, nts, terms, stream)
                : launch_lp_terms<__bf16, true>(p, a.degree, nts, terms, stream);
  }
  return fp16 ? launch_lp_terms<_Float16, false>(p, a.degree, nts, terms, stream)
              : launch_lp_terms<__bf16, false>(p, a.degree, nts, terms, stream);
}

}  // namespace mls
