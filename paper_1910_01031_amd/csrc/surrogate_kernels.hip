// Learned surrogate forecast: six 3x3 periodic convolutions (3 -> 48 x5 -> 3) in BF16 on
// the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), its backward pass,
// MSE loss, Adam and the mass-drift guard.
//
// Convolution as an implicit GEMM: M = output cells (16 consecutive cells of one row per
// MFMA tile), N = output channels (tiles of 16), K = 9 taps x input channels (ordered
// k = tap * C_in + c, tap = 3 ky + kx, padded to a multiple of 32).  Fragment layout of
// v_mfma_f32_16x16x32_bf16: lane l holds row (l % 16) of A and column (l % 16) of B with
// K elements 8 (l / 16) .. 8 (l / 16) + 7, and D rows 4 (l / 16) .. +3 of column l % 16.
// Weights are stored transposed, Wt[n][k] (bf16), so a lane reads its 8 K values as one
// 16-byte load; activations are NHWC bf16 so 8 consecutive channels of one tap are one
// 16-byte load (C_in multiple of 8) or gathered element by element (C_in = 3).
#include <cstdlib>
#include <type_traits>

#include "internal.hpp"

namespace iewpf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Two floats -> a packed pair of bf16 (a in the low half), rounded to nearest even by the
// hardware conversion (v_cvt_pk_bf16_f32): the same bits as f2bf for every non-NaN value.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  bf16x2 v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, v);
}

}  // namespace

namespace {

constexpr int kMT = 2;  // 16-cell M tiles per wave

template <int IN>
__device__ __forceinline__ bf16x8 load_a(const ConvArgs& A, int b, int y, int x, int k0) {
  bf16x8 v;
  if (IN == kInNhwcVec) {
    if (k0 >= A.K) {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.0f;
      return v;
    }
    const int tap = k0 / A.cin, c0 = k0 - tap * A.cin;
    const int ys = wrapc(y + tap / 3 - 1, A.H), xs = wrapc(x + tap % 3 - 1, A.W);
    const uint16_t* p = static_cast<const uint16_t*>(A.in) +
                        (((size_t)b * A.H + ys) * A.W + xs) * A.cin + c0;
    const uint4 raw = *reinterpret_cast<const uint4*>(p);
    v = __builtin_bit_cast(bf16x8, raw);
    return v;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + i;
      float f = 0.0f;
      if (k < A.K) {
        const int tap = k / A.cin, c = k - tap * A.cin;
        const int ys = wrapc(y + tap / 3 - 1, A.H), xs = wrapc(x + tap % 3 - 1, A.W);
        if (IN == kInStateNorm) {
          const float* st = static_cast<const float*>(A.in);
          const float val = st[(((size_t)b * 3 + c) * A.H + ys) * A.W + xs];
          f = bf2f(f2bf((val - A.mu[c]) * A.isig[c]));
        } else {
          const uint16_t* q = static_cast<const uint16_t*>(A.in);
          f = bf2f(q[(((size_t)b * A.H + ys) * A.W + xs) * A.cin + c]);
        }
      }
      v[i] = (__bf16)f;
    }
    return v;
  }
}

// Per-channel moments of training pairs (x, t) [B][3][HW]: workgroup (g, c) sums x, x^2,
// t - x, (t - x)^2 of channel c over its slice (images and cells strided by the grid) in
// float64; part[c][g][4].
constexpr int kStatBlocks = 64;
__global__ __launch_bounds__(256) void channel_moments_kernel(const float* __restrict__ x,
                                                              const float* __restrict__ t, int B,
                                                              int hw, double* __restrict__ part) {
  __shared__ double sh[4][256];
  const int c = blockIdx.y, g = blockIdx.x;
  const size_t n = (size_t)B * hw;
  double a = 0.0, a2 = 0.0, d = 0.0, d2 = 0.0;
  for (size_t e = (size_t)g * 256 + threadIdx.x; e < n; e += (size_t)kStatBlocks * 256) {
    const size_t b = e / hw, r = e - b * hw;
    const size_t o = (b * 3 + c) * hw + r;
    const double xv = x[o], dv = (double)t[o] - xv;
    a += xv;
    a2 += xv * xv;
    d += dv;
    d2 += dv * dv;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = a2;
  sh[2][threadIdx.x] = d;
  sh[3][threadIdx.x] = d2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[((size_t)c * kStatBlocks + g) * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// The parts summed in a fixed order; mean, standard deviation (n - 1 in the denominator) of
// x plus 1e-6, and of t - x plus 1e-9 (guards against constant channels):
// out = {mu[3], sigma[3], scale[3]}.
__global__ void channel_moments_finish_kernel(const double* __restrict__ part, double n,
                                              double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= 3) return;
  double a = 0.0, a2 = 0.0, d = 0.0, d2 = 0.0;
  for (int g = 0; g < kStatBlocks; ++g) {
    const double* p = part + ((size_t)c * kStatBlocks + g) * 4;
    a += p[0];
    a2 += p[1];
    d += p[2];
    d2 += p[3];
  }
  const double m = a / n, md = d / n;
  out[c] = m;
  out[3 + c] = sqrt(fmax(a2 - n * m * m, 0.0) / (n - 1.0)) + 1e-6;
  out[6 + c] = sqrt(fmax(d2 - n * md * md, 0.0) / (n - 1.0)) + 1e-9;
}

template <int IN, int OUT, int NT>
__global__ __launch_bounds__(256) void conv3x3_mfma_kernel(ConvArgs A, int total_waves) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave >= total_waves) return;
  const int xt = (A.W + 16 * kMT - 1) / (16 * kMT);
  const int b = wave / (A.H * xt);
  const int r = wave - b * A.H * xt;
  const int y = r / xt;
  const int x0 = (r - y * xt) * 16 * kMT;
  const int row = lane & 15, kq = lane >> 4;
  int xa[kMT];  // A-operand cell of this lane per M tile (cells past the row end wrap; unused)
#pragma unroll
  for (int m = 0; m < kMT; ++m) xa[m] = (x0 + m * 16 + row) % A.W;
  f32x4 acc[kMT][NT];
#pragma unroll
  for (int m = 0; m < kMT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int nchunks = A.Kpad / 32;
  for (int kc = 0; kc < nchunks; ++kc) {
    const int k0 = kc * 32 + kq * 8;
    bf16x8 bfr[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const uint16_t* p = A.wt + (size_t)(t * 16 + row) * A.Kpad + k0;
      bfr[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
    }
#pragma unroll
    for (int m = 0; m < kMT; ++m) {
      const bf16x8 afr = load_a<IN>(A, b, y, xa[m], k0);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[t], acc[m][t], 0, 0, 0);
    }
  }
  // epilogue: lane holds cells 4 kq .. 4 kq + 3 of column n = 16 t + row
#pragma unroll
  for (int m = 0; m < kMT; ++m) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 16 + row;
      if (n >= A.cout) continue;
      const float bn = A.bias ? A.bias[n] : 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int x = x0 + m * 16 + kq * 4 + q;
        if (x >= A.W) continue;
        const size_t cell = ((size_t)b * A.H + y) * A.W + x;
        const float v = acc[m][t][q] + bn;
        if (OUT == kOutReluBf16) {
          static_cast<uint16_t*>(A.out)[cell * A.cout + n] = f2bf(fmaxf(v, 0.0f));
        } else if (OUT == kOutF32) {
          static_cast<float*>(A.out)[cell * A.cout + n] = v;
        } else if (OUT == kOutMaskBf16) {
          const bool on = bf2f(A.mask[cell * A.cout + n]) > 0.0f;
          static_cast<uint16_t*>(A.out)[cell * A.cout + n] = f2bf(on ? v : 0.0f);
        } else {  // residual into the state: psi' = psi + s (net)
          const size_t o = (((size_t)b * 3 + n) * A.H + y) * A.W + x;
          static_cast<float*>(A.out)[o] = A.state_in[o] + A.s[n] * v;
        }
      }
    }
  }
}

// Convolutions of the network as a persistent, LDS-tiled implicit GEMM (every forward layer
// and the 48 -> 48 input gradients of the backward pass).  A workgroup of kTH waves owns a
// tile of kTH output rows x kTW columns of one image.  The (kTH + 2) x (kTW + 2) input
// pixels (periodic wrap) sit in LDS, as do the layer's weights (loaded once per workgroup);
// every wave computes one output row as kTW / 16 pixel tiles x NT channel tiles of
// v_mfma_f32_16x16x32_bf16.  The operands are swapped with respect to the generic kernel
// (A = weights, rows = output channels; B = pixels), so a lane ends with 4 consecutive
// channels of one pixel.  While a tile is computed, the next tile's input is already being
// fetched into registers; it is written to LDS between two barriers.
//   CIN = 48: hidden-layer input, bf16 NHWC, K = 9 x 48 (14 chunks of 32), k = 48 tap + c.
//   CIN = 8:  the normalised state (3 channels zero-padded to 8), K = 9 x 8 (3 chunks),
//             k = 8 tap + c; the weights are re-laid from their k = 3 tap + c form.
// LDS strides.  A 16-byte LDS read (ds_read_b128) is served 32 lanes at a time, and
// measured bank conflicts on gfx950 fit 128 banks of 4 bytes: the 32 lanes (16 rows x 2
// K-quads 16 bytes apart) are conflict-free when the row stride in 4-byte words is 8 x odd
// modulo 128.  Pixel stride: 48 channels = 24 words (conflict-free unpadded); weight rows:
// the 432 stored K values = 216 words (lanes past K take zero fragments instead of reading),
// and 56 words for the 96 (zero-padded) K values of the 8-channel input.
template <int CIN>
struct TileGeom {
  static constexpr int CP = CIN;                     // LDS pixel stride (bf16)
  static constexpr int CHUNKS = CIN == 48 ? 14 : 3;  // K chunks of 32
  static constexpr int KP = CHUNKS * 32;             // padded K
  static constexpr int KW = CIN == 48 ? 432 : 96;    // K values stored per weight row
  static constexpr int WS = CIN == 48 ? 432 : 112;   // LDS weight row stride (bf16)
  static constexpr int VPP = CIN / 8;                // 16-byte vectors per pixel (NHWC input)
};
__device__ __forceinline__ int wrapm(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}
// A tile's input coordinate (from one before the image to one tile past its end) wrapped onto
// [0, n): one correction each way covers images larger than a tile; the remainder, which
// costs a division, runs only for the lanes of smaller images.
__device__ __forceinline__ int wrap_tile(int i, int n) {
  if (i < 0) i += n;
  if (i >= n) i -= n;
  if (i < 0 || i >= n) i = wrapm(i, n);
  return i;
}

template <int kTH, int kTW>
__device__ __forceinline__ void tile_origin(int t, int xt, int yt, int& b, int& y0, int& x0) {
  b = t / (yt * xt);
  const int r = t - b * yt * xt;
  y0 = (r / xt) * kTH;
  x0 = (r - (r / xt) * xt) * kTW;
}

template <int CIN, int NT, int kTH, int kTW>
constexpr int tile_lds_bytes() {  // input tile, weights, then the NT x 16 bias values (float)
  return 2 * ((kTH + 2) * (kTW + 2) * TileGeom<CIN>::CP + NT * 16 * TileGeom<CIN>::WS) +
         4 * NT * 16;
}

// MFMA part of one tile for output row `wave` of the tile held in LDS: acc = W x inputs.
template <int CIN, int NT, int kTW>
__device__ __forceinline__ void tile_mfma(const uint16_t* tile, const uint16_t* wl, int wave,
                                          int row, int kq, f32x4 (&acc)[NT][kTW / 16]) {
  using G = TileGeom<CIN>;
  constexpr int kTM = kTW / 16;
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int m = 0; m < kTM; ++m) acc[q][m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kc = 0; kc < G::CHUNKS; ++kc) {
    const int k = kc * 32 + kq * 8;
    int tap, c0;
    if (CIN == 48) {
      tap = k / 48;
      c0 = k - tap * 48;
      if (k >= 9 * 48) {  // padding: zero weights times valid (finite) activations
        tap = 8;
        c0 = 0;
      }
    } else {
      tap = k / 8;
      c0 = 0;
      if (tap > 8) tap = 8;  // padding taps: zero weights
    }
    const int dy = tap / 3, dx = tap - dy * 3;
    const uint16_t* base = tile + ((wave + dy) * (kTW + 2) + dx + row) * G::CP + c0;
    bf16x8 afr[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      u32x4 w = u32x4{0u, 0u, 0u, 0u};
      if (kc * 32 + 32 <= G::KW || k < G::KW)  // the first test is compile-time
        w = *reinterpret_cast<const u32x4*>(wl + (q * 16 + row) * G::WS + k);
      afr[q] = __builtin_bit_cast(bf16x8, w);
    }
#pragma unroll
    for (int m = 0; m < kTM; ++m) {
      const bf16x8 bfr =
          __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(base + m * 16 * G::CP));
#pragma unroll
      for (int q = 0; q < NT; ++q)
        acc[q][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[q], bfr, acc[q][m], 0, 0, 0);
    }
  }
}

// The bias values of this lane's output channels (16 q + 4 kq .. + 3), loaded once.
template <int NT>
__device__ __forceinline__ void lane_bias(const ConvArgs& A, int kq, float (&bias)[NT][4]) {
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int n = NT == 1 ? e : q * 16 + kq * 4 + e;
      bias[q][e] = (A.bias && n < A.cout) ? A.bias[n] : 0.0f;
    }
  // The loads are waited for here, once.  Left to their first use inside the persistent tile
  // loop, the wait there would also cover every load issued after them (the next tile's
  // prefetch), on every tile.
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) asm volatile("" ::"v"(bias[q][e]));
}

// Epilogue of one tile row: bias, activation / mask / residual, stores.
template <int NT, int OUT, int kTM>
__device__ __forceinline__ void tile_store(const ConvArgs& A, const f32x4 (&acc)[NT][kTM],
                                           const float (&bias)[NT][4], int b, int y, int x0,
                                           int row, int kq, int cols = 16 * kTM) {
  // lane: pixel x0 + 16 m + row, channels 16 q + 4 kq .. + 3; only the tile's first `cols`
  // columns are stored
#pragma unroll
  for (int m = 0; m < kTM; ++m) {
    const int x = x0 + m * 16 + row;
    if (x >= A.W || m * 16 + row >= cols) continue;
    const size_t cell = ((size_t)b * A.H + y) * A.W + x;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int n0 = q * 16 + kq * 4;
      if (OUT == kOutReluBf16) {
        float r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = fmaxf(acc[q][m][e] + bias[q][e], 0.0f);
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(A.out) + cell * A.cout + n0) =
            make_uint2(pack_bf16x2(r[0], r[1]), pack_bf16x2(r[2], r[3]));
      } else if (OUT == kOutMaskBf16) {
        const uint2 mk = *reinterpret_cast<const uint2*>(A.mask + cell * A.cout + n0);
        uint32_t h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float v = acc[q][m][e] + bias[q][e];
          const uint32_t word = e < 2 ? mk.x : mk.y;
          const uint16_t me = (uint16_t)(e & 1 ? word >> 16 : word & 0xFFFFu);
          h[e] = f2bf(bf2f(me) > 0.0f ? v : 0.0f);
        }
        *reinterpret_cast<uint2*>(static_cast<uint16_t*>(A.out) + cell * A.cout + n0) =
            make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
      } else if (kq == 0) {  // NT == 1: channels 0..2 of the state
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const float v = acc[q][m][e] + bias[q][e];
          if (OUT == kOutF32) {
            static_cast<float*>(A.out)[cell * 3 + e] = v;
          } else {  // residual into the state: psi' = psi + s (net)
            const size_t o = (((size_t)b * 3 + e) * A.H + y) * A.W + x;
            static_cast<float*>(A.out)[o] = A.state_in[o] + A.s[e] * v;
          }
        }
      }
    }
  }
}

// The 48 -> 3 layer (NT = 1) is bound by memory latency, not by the matrix cores: its
// 32-column tiles are asked to fit more waves per SIMD, so that more workgroups (more tiles in
// flight) share a compute unit: three of 8 rows (6 waves per SIMD) or two of 16 rows (8).
template <int NT, int kTH, int kTW>
constexpr int conv_min_waves() {
  return (NT == 1 && kTW == 32) ? (kTH == 8 ? 6 : 8) : 1;
}
template <int CIN, int NT, int IN, int OUT, int kTH, int kTW>
__global__ __launch_bounds__(64 * kTH, (conv_min_waves<NT, kTH, kTW>())) void conv_tile_kernel(
    ConvArgs A, int ntiles) {
  constexpr int kTM = kTW / 16;
  constexpr int kTThreads = 64 * kTH;
  using G = TileGeom<CIN>;
  constexpr int kPix = (kTH + 2) * (kTW + 2);
  constexpr int kTileElems = kPix * G::CP;
  extern __shared__ __align__(16) uint16_t lds[];
  uint16_t* tile = lds;
  uint16_t* wl = lds + kTileElems;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;

  // weights -> LDS, [NT * 16][WS]
  for (int i = threadIdx.x; i < NT * 16 * (G::KW / 8); i += kTThreads) {
    const int n = i / (G::KW / 8), kv = i - n * (G::KW / 8);
    uint4 v;
    if (CIN == 48) {
      v = *reinterpret_cast<const uint4*>(A.wt + (size_t)n * A.Kpad + kv * 8);
    } else {  // kv = tap; stored layout k = 3 tap + c
      uint32_t e0 = 0, e1 = 0;
      if (kv < 9) {
        const uint16_t* src = A.wt + (size_t)n * A.Kpad + kv * 3;
        e0 = (uint32_t)src[0] | ((uint32_t)src[1] << 16);
        e1 = (uint32_t)src[2];
      }
      v = make_uint4(e0, e1, 0u, 0u);
    }
    *reinterpret_cast<uint4*>(wl + n * G::WS + kv * 8) = v;
  }

  // bias -> LDS, read by the epilogue of every tile (so the bias values hold no registers
  // across the tile loop)
  float* lbias = reinterpret_cast<float*>(wl + NT * 16 * G::WS);
  for (int i = threadIdx.x; i < NT * 16; i += kTThreads)
    lbias[i] = (A.bias && i < A.cout) ? A.bias[i] : 0.0f;

  const int xt = (A.W + kTW - 1) / kTW, yt = (A.H + kTH - 1) / kTH;

  // registers holding the next tile's input
  constexpr int kVecs = IN == kInStateNorm ? kPix : kPix * G::VPP;
  constexpr int kPer = (kVecs + kTThreads - 1) / kTThreads;
  u32x4 pre[IN == kInStateNorm ? 1 : kPer];
  float pf[IN == kInStateNorm ? kPer : 1][3];
  auto fetch = [&](int tn) {  // tile tn's input -> registers
    int b, y0, x0;
    tile_origin<kTH, kTW>(tn, xt, yt, b, y0, x0);
    // wave-uniform: the tile and its halo lie inside the image, no coordinate wraps
    const bool inside = y0 >= 1 && y0 + kTH + 1 <= A.H && x0 >= 1 && x0 + kTW + 1 <= A.W;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int v = threadIdx.x + i * kTThreads;
      if (v < kVecs) {
        // the image's base is wave-uniform, the pixel's offset 32-bit
        if (IN == kInStateNorm) {
          const int rr = v / (kTW + 2), cc = v - rr * (kTW + 2);
          const int ys = wrap_tile(y0 - 1 + rr, A.H), xs = wrap_tile(x0 - 1 + cc, A.W);
          const size_t plane = (size_t)A.H * A.W;
          const float* img = static_cast<const float*>(A.in) + (size_t)b * 3 * plane;
          const unsigned off = static_cast<unsigned>(ys) * A.W + xs;
          pf[i][0] = img[off];
          pf[i][1] = (img + plane)[off];
          pf[i][2] = (img + 2 * plane)[off];
        } else {
          const int pix = v / G::VPP, cv = v - pix * G::VPP;
          const int rr = pix / (kTW + 2), cc = pix - rr * (kTW + 2);
          int ys = y0 - 1 + rr, xs = x0 - 1 + cc;
          if (!inside) {
            ys = wrap_tile(ys, A.H);
            xs = wrap_tile(xs, A.W);
          }
          const uint16_t* img = static_cast<const uint16_t*>(A.in) + (size_t)b * A.H * A.W * CIN;
          const unsigned off = (static_cast<unsigned>(ys) * A.W + xs) * CIN + cv * 8;
          pre[i] = *reinterpret_cast<const u32x4*>(img + off);
        }
      }
    }
  };
  auto commit = [&](uint16_t* dst) {  // registers -> LDS tile
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int v = threadIdx.x + i * kTThreads;
      if (v < kVecs) {
        if (IN == kInStateNorm) {
          uint32_t h[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) h[c] = f2bf((pf[i][c] - A.mu[c]) * A.isig[c]);
          *reinterpret_cast<uint4*>(dst + v * G::CP) = make_uint4(h[0] | (h[1] << 16), h[2], 0u, 0u);
        } else {
          const int pix = v / G::VPP, cv = v - pix * G::VPP;
          *reinterpret_cast<u32x4*>(dst + pix * G::CP + cv * 8) = pre[i];
        }
      }
    }
  };
  auto compute = [&](const uint16_t* src, int t) {
    int b, y0, x0;
    tile_origin<kTH, kTW>(t, xt, yt, b, y0, x0);
    const int y = y0 + wave;
    if (y < A.H) {  // wave-uniform
      f32x4 acc[NT][kTM];
      tile_mfma<CIN, NT, kTW>(src, wl, wave, row, kq, acc);
      // this lane's bias values: channels 16 q + 4 kq .. + 3 (NT = 1: channels 0 .. 3)
      float bias[NT][4];
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const float4 bv = *reinterpret_cast<const float4*>(lbias + (NT == 1 ? 0 : q * 16 + kq * 4));
        bias[q][0] = bv.x;
        bias[q][1] = bv.y;
        bias[q][2] = bv.z;
        bias[q][3] = bv.w;
      }
      tile_store<NT, OUT, kTM>(A, acc, bias, b, y, x0, row, kq);
    }
  };

  // Iteration t: write tile t (fetched in the previous iteration) to LDS, start fetching
  // tile t + gridDim.x, compute tile t.  The first fetch is peeled off the loop (the grid is
  // at most ntiles workgroups), so every fetch follows a commit that has waited for the
  // previous one's loads and the fetch's own loads are not waited for one by one.
  int t = (int)blockIdx.x;
  fetch(t);
  for (; t < ntiles; t += gridDim.x) {
    const int tn = t + (int)gridDim.x;
    __syncthreads();  // weights written / the previous tile's LDS reads are done
    commit(tile);
    __syncthreads();
    if (tn < ntiles) fetch(tn);  // in flight during the MFMAs below
    compute(tile, t);
  }
}

// Two consecutive layers in one pass (forward only): layer A (C_in -> 48, ReLU, BF16) over a
// (kPairTH + 2) x 32 region into an LDS tile, then layer B (48 -> 16 NT_B) over the kPairTH x
// kPairTW output tile from it, so A's activation never goes to HBM.  Both layers use
// tile_mfma (the same fragments, K order and accumulation as the one-layer kernel) and the
// same epilogue arithmetic, so the outputs equal the layer-by-layer pass bit for bit.
// Geometry: input tile (kPairTH + 4) x 34 pixels from (y0 - 2, x0 - 2), intermediate tile
// (kPairTH + 2) rows x 34 pixels (32 written; the two past them feed only output columns 30
// and 31, which are computed and dropped), output tile kPairTH x kPairTW (wave w computes
// intermediate row w, then output row w for w < kPairTH).
constexpr int kPairTW = 30, kPairCols = 32;

template <int CIN, int NT>
__device__ __forceinline__ void weights_to_lds(const ConvArgs& A, uint16_t* wl, int nthreads) {
  using G = TileGeom<CIN>;
  for (int i = threadIdx.x; i < NT * 16 * (G::KW / 8); i += nthreads) {
    const int n = i / (G::KW / 8), kv = i - n * (G::KW / 8);
    uint4 v;
    if (CIN == 48) {
      v = *reinterpret_cast<const uint4*>(A.wt + (size_t)n * A.Kpad + kv * 8);
    } else {  // kv = tap; stored layout k = 3 tap + c
      uint32_t e0 = 0, e1 = 0;
      if (kv < 9) {
        const uint16_t* src = A.wt + (size_t)n * A.Kpad + kv * 3;
        e0 = (uint32_t)src[0] | ((uint32_t)src[1] << 16);
        e1 = (uint32_t)src[2];
      }
      v = make_uint4(e0, e1, 0u, 0u);
    }
    *reinterpret_cast<uint4*>(wl + n * G::WS + kv * 8) = v;
  }
}

template <int CIN_A, int kPairTH>
constexpr int pair_lds_bytes(int nt_b) {
  return 2 * ((kPairTH + 4) * (kPairCols + 2) * TileGeom<CIN_A>::CP +
              (kPairTH + 2) * (kPairCols + 2) * 48 + 48 * TileGeom<CIN_A>::WS +
              nt_b * 16 * TileGeom<48>::WS);
}

template <int CIN_A, int IN_A, int NT_B, int OUT_B, int kPairTH>
__global__ __launch_bounds__(64 * (kPairTH + 2)) void conv_pair_kernel(ConvArgs LA, ConvArgs LB,
                                                                       int ntiles) {
  constexpr int kPairThreads = 64 * (kPairTH + 2);
  using GA = TileGeom<CIN_A>;
  using GB = TileGeom<48>;
  constexpr int kInW = kPairCols + 2;                   // 34 pixels per tile row
  constexpr int kInPix = (kPairTH + 4) * kInW;
  extern __shared__ __align__(16) uint16_t lds[];
  uint16_t* tin = lds;                                  // [(TH + 4) * 34][CP_A]
  uint16_t* tmid = tin + kInPix * GA::CP;               // [(TH + 2) * 34][48]
  uint16_t* wa = tmid + (kPairTH + 2) * kInW * 48;      // [48][WS_A]
  uint16_t* wb = wa + 48 * GA::WS;                      // [16 NT_B][WS_B]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  weights_to_lds<CIN_A, 3>(LA, wa, kPairThreads);
  weights_to_lds<48, NT_B>(LB, wb, kPairThreads);
  const int xt = (LB.W + kPairTW - 1) / kPairTW, yt = (LB.H + kPairTH - 1) / kPairTH;
  float bias_a[3][4], bias_b[NT_B][4];
  lane_bias<3>(LA, kq, bias_a);
  lane_bias<NT_B>(LB, kq, bias_b);

  constexpr int kVecs = IN_A == kInStateNorm ? kInPix : kInPix * GA::VPP;
  constexpr int kPer = (kVecs + kPairThreads - 1) / kPairThreads;
  u32x4 pre[IN_A == kInStateNorm ? 1 : kPer];
  float pf[IN_A == kInStateNorm ? kPer : 1][3];
  auto origin = [&](int t, int& b, int& y0, int& x0) {
    b = t / (yt * xt);
    const int r = t - b * yt * xt;
    y0 = (r / xt) * kPairTH;
    x0 = (r - (r / xt) * xt) * kPairTW;
  };
  auto fetch = [&](int tn) {  // tile tn's input (rows y0 - 2 .., columns x0 - 2 ..) -> registers
    int b, y0, x0;
    origin(tn, b, y0, x0);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int v = threadIdx.x + i * kPairThreads;
      if (v < kVecs) {
        // the image's base is wave-uniform, the pixel's offset 32-bit
        if (IN_A == kInStateNorm) {
          const int rr = v / kInW, cc = v - rr * kInW;
          const int ys = wrap_tile(y0 - 2 + rr, LA.H), xs = wrap_tile(x0 - 2 + cc, LA.W);
          const size_t plane = (size_t)LA.H * LA.W;
          const float* img = static_cast<const float*>(LA.in) + (size_t)b * 3 * plane;
          const unsigned off = static_cast<unsigned>(ys) * LA.W + xs;
          pf[i][0] = img[off];
          pf[i][1] = (img + plane)[off];
          pf[i][2] = (img + 2 * plane)[off];
        } else {
          const int pix = v / GA::VPP, cv = v - pix * GA::VPP;
          const int rr = pix / kInW, cc = pix - rr * kInW;
          const int ys = wrap_tile(y0 - 2 + rr, LA.H), xs = wrap_tile(x0 - 2 + cc, LA.W);
          const uint16_t* img =
              static_cast<const uint16_t*>(LA.in) + (size_t)b * LA.H * LA.W * CIN_A;
          const unsigned off = (static_cast<unsigned>(ys) * LA.W + xs) * CIN_A + cv * 8;
          pre[i] = *reinterpret_cast<const u32x4*>(img + off);
        }
      }
    }
  };
  auto commit = [&]() {  // registers -> LDS input tile
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int v = threadIdx.x + i * kPairThreads;
      if (v < kVecs) {
        if (IN_A == kInStateNorm) {
          uint32_t h[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) h[c] = f2bf((pf[i][c] - LA.mu[c]) * LA.isig[c]);
          *reinterpret_cast<uint4*>(tin + v * GA::CP) = make_uint4(h[0] | (h[1] << 16), h[2], 0u, 0u);
        } else {
          const int pix = v / GA::VPP, cv = v - pix * GA::VPP;
          *reinterpret_cast<u32x4*>(tin + pix * GA::CP + cv * 8) = pre[i];
        }
      }
    }
  };
  auto compute = [&](int t) {
    int b, y0, x0;
    origin(t, b, y0, x0);
    {  // layer A: intermediate row `wave` (global row y0 - 1 + wave, wrapped), 32 columns
      f32x4 acc[3][2];
      tile_mfma<CIN_A, 3, kPairCols>(tin, wa, wave, row, kq, acc);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int n0 = q * 16 + kq * 4;
          float r[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) r[e] = fmaxf(acc[q][m][e] + bias_a[q][e], 0.0f);
          *reinterpret_cast<uint2*>(tmid + (wave * kInW + m * 16 + row) * 48 + n0) =
              make_uint2(pack_bf16x2(r[0], r[1]), pack_bf16x2(r[2], r[3]));
        }
    }
    __syncthreads();
    const int y = y0 + wave;
    if (wave < kPairTH && y < LB.H) {  // layer B: output row `wave`, columns x0 .. x0 + 29
      f32x4 acc[NT_B][2];
      tile_mfma<48, NT_B, kPairCols>(tmid, wb, wave, row, kq, acc);
      tile_store<NT_B, OUT_B, 2>(LB, acc, bias_b, b, y, x0, row, kq, kPairTW);
    }
  };
  // the first fetch peeled off the loop, as in conv_tile_kernel
  int t = (int)blockIdx.x;
  fetch(t);
  for (; t < ntiles; t += gridDim.x) {
    const int tn = t + (int)gridDim.x;
    __syncthreads();  // weights written / the previous tile's LDS reads are done
    commit();
    __syncthreads();
    if (tn < ntiles) fetch(tn);  // in flight during the MFMAs below
    compute(t);
  }
}

// Weight gradient of one layer over a chunk of cells: dW[n][k] = sum_cells g[cell][n] *
// a(cell shifted by tap(k))[c(k)], as MFMA with M = n (16-tiles), N = k (16-tiles),
// K = cells (32 per step).  Partial sums per chunk go to part[chunk][Npad][Kpad].
template <int IN>
__global__ __launch_bounds__(256) void wgrad_mfma_kernel(ConvArgs A, const uint16_t* __restrict__ g,
                                                         int gch, int cells_per_chunk,
                                                         float* __restrict__ part, int total_waves) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave >= total_waves) return;
  const int ktiles = A.Kpad / 16;
  const int chunk = wave / ktiles;
  const int ktile = wave - chunk * ktiles;
  const int row = lane & 15, kq = lane >> 4;
  const int ncells = A.B * A.H * A.W;
  const int c_begin = chunk * cells_per_chunk;
  const int c_end = min(c_begin + cells_per_chunk, ncells);
  const int mtiles = A.Npad / 16;
  f32x4 acc[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int k = ktile * 16 + row;  // B column of this lane
  int tap = 0, c = 0;
  if (k < A.K) {
    tap = k / A.cin;
    c = k - tap * A.cin;
  }
  for (int p0 = c_begin; p0 < c_end; p0 += 32) {
    bf16x8 bfr;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int p = p0 + kq * 8 + i;
      float f = 0.0f;
      if (p < c_end && k < A.K) {
        const int b = p / (A.H * A.W);
        const int rr = p - b * A.H * A.W;
        const int yy = rr / A.W, xx = rr - yy * A.W;
        const int ys = wrapc(yy + tap / 3 - 1, A.H), xs = wrapc(xx + tap % 3 - 1, A.W);
        if (IN == kInStateNorm) {
          const float* st = static_cast<const float*>(A.in);
          f = bf2f(f2bf((st[(((size_t)b * 3 + c) * A.H + ys) * A.W + xs] - A.mu[c]) * A.isig[c]));
        } else {
          const uint16_t* q = static_cast<const uint16_t*>(A.in);
          f = bf2f(q[(((size_t)b * A.H + ys) * A.W + xs) * A.cin + c]);
        }
      }
      bfr[i] = (__bf16)f;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (t >= mtiles) break;
      bf16x8 afr;
      const int n = t * 16 + row;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = p0 + kq * 8 + i;
        afr[i] = (__bf16)((p < c_end && n < gch) ? bf2f(g[(size_t)p * gch + n]) : 0.0f);
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr, acc[t], 0, 0, 0);
    }
  }
  // D: rows n = 16 t + 4 kq + q, column k
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t >= mtiles) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = t * 16 + kq * 4 + q;
      part[((size_t)chunk * A.Npad + n) * A.Kpad + k] = acc[t][q];
    }
  }
}

// bias gradient partials: part[chunk][n] = sum over the chunk's cells of g[cell][n]
__global__ void bgrad_kernel(const uint16_t* __restrict__ g, int gch, int ncells, int cells_per_chunk,
                             float* __restrict__ part) {
  const int chunk = blockIdx.x;
  const int n = threadIdx.x;
  if (n >= gch) return;
  const int c0 = chunk * cells_per_chunk, c1 = min(c0 + cells_per_chunk, ncells);
  float s = 0.0f;
  for (int p = c0; p < c1; ++p) s += bf2f(g[(size_t)p * gch + n]);
  part[(size_t)chunk * gch + n] = s;
}

// Sum partials over chunks in fixed order into the FP32 gradient of one layer
// ([cout][cin][3][3] then [cout]).
__global__ void reduce_grads_kernel(const float* __restrict__ wpart, const float* __restrict__ bpart,
                                    int nchunks, int cin, int cout, int Kpad, int Npad,
                                    float* __restrict__ gw, float* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = cout * cin * 9;
  if (i < nw) {
    const int n = i / (cin * 9);
    const int rem = i - n * cin * 9;
    const int c = rem / 9, tap = rem - c * 9;
    const int k = tap * cin + c;
    float s = 0.0f;
    for (int q = 0; q < nchunks; ++q) s += wpart[((size_t)q * Npad + n) * Kpad + k];
    gw[i] = s;
  } else if (i < nw + cout) {
    const int n = i - nw;
    float s = 0.0f;
    for (int q = 0; q < nchunks; ++q) s += bpart[(size_t)q * cout + n];
    gb[n] = s;
  }
}

// MSE of the network output y (float [cells][3]) against the normalised increment
// (target - state)/s: per-block partial losses and g = bf16(2 (y - t) / n).
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ st_in,
                           const float* __restrict__ st_tgt, int B, int H, int W, float s0, float s1,
                           float s2, uint16_t* __restrict__ g, float* __restrict__ lpart) {
  __shared__ float sh[256];
  const int ncells = B * H * W;
  const float inv_n = 1.0f / (3.0f * ncells);
  const float s[3] = {s0, s1, s2};
  float acc = 0.0f;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < ncells; p += gridDim.x * blockDim.x) {
    const int b = p / (H * W), rr = p - b * H * W;
    for (int ch = 0; ch < 3; ++ch) {
      const size_t o = ((size_t)b * 3 + ch) * H * W + rr;
      const float t = (st_tgt[o] - st_in[o]) / s[ch];
      const float d = y[(size_t)p * 3 + ch] - t;
      acc += d * d;
      g[(size_t)p * 3 + ch] = f2bf(2.0f * d * inv_n);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0] * inv_n;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Forward and transposed (input-gradient) bf16 layouts of one layer from its FP32 master
// weights w[cout][cin][3][3]: wf[n][tap cin + c] = w[n][c][tap];
// wd[c][tap' cout + n] = w[n][c][8 - tap'] (spatially flipped, channels swapped).
__global__ void prep_weights_kernel(const float* __restrict__ w, int cin, int cout, int Kf, int Npf,
                                    int Kd, int Npd, uint16_t* __restrict__ wf,
                                    uint16_t* __restrict__ wd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = Npf * Kf, nd = wd ? Npd * Kd : 0;
  if (i < nf) {
    const int n = i / Kf, k = i - n * Kf;
    float v = 0.0f;
    if (n < cout && k < 9 * cin) {
      const int tap = k / cin, c = k - tap * cin;
      v = w[((size_t)n * cin + c) * 9 + tap];
    }
    wf[i] = f2bf(v);
  } else if (i < nf + nd) {
    const int j = i - nf;
    const int c = j / Kd, k = j - c * Kd;
    float v = 0.0f;
    if (c < cin && k < 9 * cout) {
      const int tap = k / cout, n = k - tap * cout;
      v = w[((size_t)n * cin + c) * 9 + (8 - tap)];
    }
    wd[j] = f2bf(v);
  }
}

// Per-particle relative mass drift |sum(H + eta') - sum(H + eta)| / sum(H + eta) in FP64;
// flags[i] = drift > tol.
__global__ void mass_drift_kernel(const float* __restrict__ before, const float* __restrict__ after,
                                  int ncell, double H, double tol, double* __restrict__ drift,
                                  int32_t* __restrict__ flags) {
  __shared__ double sa[256], sb[256];
  const int i = blockIdx.x;
  const float* e0 = before + (size_t)i * 3 * ncell;
  const float* e1 = after + (size_t)i * 3 * ncell;
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < ncell; c += 256) {
    a += (double)e0[c];
    b += (double)e1[c];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m0 = H * ncell + sa[0], m1 = H * ncell + sb[0];
    const double d = fabs(m1 - m0) / m0;
    drift[i] = d;
    flags[i] = (d > tol || !isfinite(d)) ? 1 : 0;
  }
}

// one wave: the flags summed lane by lane, then across the wave
__global__ __launch_bounds__(64) void count_flags_kernel(const int32_t* __restrict__ flags, int n,
                                                         int32_t* __restrict__ out) {
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 64) c += flags[i] != 0 ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (threadIdx.x == 0) out[0] = c;
}

// grid (chunks, particles): particle blockIdx.y copied if flagged
__global__ __launch_bounds__(256) void copy_flagged_kernel(const float* __restrict__ src,
                                                           float* __restrict__ dst,
                                                           const int32_t* __restrict__ flags,
                                                           size_t per) {
  const int i = blockIdx.y;
  if (flags[i] == 0) return;
  const float* a = src + (size_t)i * per;
  float* b = dst + (size_t)i * per;
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < per; k += (size_t)gridDim.x * 256)
    b[k] = a[k];
}

template <int IN, int OUT, int NT>
void launch_conv_t(const ConvArgs& A, hipStream_t s) {
  const int xt = (A.W + 16 * kMT - 1) / (16 * kMT);
  const int waves = A.B * A.H * xt;
  hipLaunchKernelGGL((conv3x3_mfma_kernel<IN, OUT, NT>), dim3((waves + 3) / 4), dim3(256), 0, s, A,
                     waves);
}

}  // namespace

static int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

template <int CIN, int NT, int IN, int OUT, int kTH, int kTW>
void launch_tile(const ConvArgs& A, hipStream_t s) {
  constexpr int bytes = tile_lds_bytes<CIN, NT, kTH, kTW>();
  constexpr int threads = 64 * kTH;
  auto* kern = conv_tile_kernel<CIN, NT, IN, OUT, kTH, kTW>;
  static int per_cu = 0;  // resident workgroups per CU (registers and LDS)
  if (per_cu == 0) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kern),
                                                     threads, bytes) != hipSuccess || n < 1)
      n = 1;
    per_cu = n;
  }
  const int ntiles = A.B * ((A.H + kTH - 1) / kTH) * ((A.W + kTW - 1) / kTW);
  const int nb = ntiles < per_cu * cu_count() ? ntiles : per_cu * cu_count();
  hipLaunchKernelGGL(kern, dim3(nb), dim3(threads), bytes, s, A, ntiles);
}

// Tile shape per layer kind (rows x columns): 0 = 8 x 32, 1 = 8 x 64, 2 = 16 x 32,
// 3 = 16 x 64.  The defaults are the fastest measured at 100 x 300 x 500 (outputs are
// identical for every shape); IEWPF_CONV_SHAPE_<kind> selects another one for timing.
int conv_shape(const char* name, int def) {
  const char* v = std::getenv(name);
  const int x = v ? std::atoi(v) : def;
  return x >= 0 && x <= 3 ? x : def;
}

template <int CIN, int NT, int IN, int OUT>
void launch_tile_shape(const ConvArgs& A, int shape, hipStream_t s) {
  switch (shape) {
    case 1: return launch_tile<CIN, NT, IN, OUT, 8, 64>(A, s);
    case 2: return launch_tile<CIN, NT, IN, OUT, 16, 32>(A, s);
    case 3: return launch_tile<CIN, NT, IN, OUT, 16, 64>(A, s);
    default: return launch_tile<CIN, NT, IN, OUT, 8, 32>(A, s);
  }
}

void launch_conv(const ConvArgs& A, int in_mode, int out_mode, hipStream_t s) {
  static const int shape_hidden = conv_shape("IEWPF_CONV_SHAPE_HIDDEN", 2);
  static const int shape_first = conv_shape("IEWPF_CONV_SHAPE_FIRST", 3);
  static const int shape_last = conv_shape("IEWPF_CONV_SHAPE_LAST", 0);
  if (in_mode == kInNhwcVec && A.cin == 48 && A.Kpad == TileGeom<48>::KP) {
    if (A.cout == 48 && A.Npad == 48 && out_mode == kOutReluBf16)
      return launch_tile_shape<48, 3, kInNhwcVec, kOutReluBf16>(A, shape_hidden, s);
    if (A.cout == 48 && A.Npad == 48 && out_mode == kOutMaskBf16)
      return launch_tile_shape<48, 3, kInNhwcVec, kOutMaskBf16>(A, shape_hidden, s);
    if (A.cout == 3 && A.Npad == 16 && out_mode == kOutResidState)
      return launch_tile_shape<48, 1, kInNhwcVec, kOutResidState>(A, shape_last, s);
    if (A.cout == 3 && A.Npad == 16 && out_mode == kOutF32)
      return launch_tile_shape<48, 1, kInNhwcVec, kOutF32>(A, shape_last, s);
  }
  if (in_mode == kInStateNorm && A.cin == 3 && A.cout == 48 && A.Npad == 48 && A.Kpad == 32 &&
      out_mode == kOutReluBf16)
    return launch_tile_shape<8, 3, kInStateNorm, kOutReluBf16>(A, shape_first, s);
  const int nt = A.Npad / 16;
#define IEWPF_CONV_CASE(I, O, T) \
  if (in_mode == I && out_mode == O && nt == T) return launch_conv_t<I, O, T>(A, s);
  IEWPF_CONV_CASE(kInStateNorm, kOutReluBf16, 3)
  IEWPF_CONV_CASE(kInNhwcVec, kOutReluBf16, 3)
  IEWPF_CONV_CASE(kInNhwcVec, kOutResidState, 1)
  IEWPF_CONV_CASE(kInNhwcVec, kOutF32, 1)
  IEWPF_CONV_CASE(kInNhwcVec, kOutMaskBf16, 3)
  IEWPF_CONV_CASE(kInNhwcSmall, kOutMaskBf16, 3)
#undef IEWPF_CONV_CASE
}

template <int CIN_A, int IN_A, int NT_B, int OUT_B, int kPairTH>
void launch_pair_t(const ConvArgs& LA, const ConvArgs& LB, hipStream_t s) {
  constexpr int bytes = pair_lds_bytes<CIN_A, kPairTH>(NT_B);
  constexpr int kPairThreads = 64 * (kPairTH + 2);
  static_assert(bytes <= 160 * 1024, "the pair's tiles and weights exceed the LDS");
  auto* kern = conv_pair_kernel<CIN_A, IN_A, NT_B, OUT_B, kPairTH>;
  static int per_cu = 0;
  if (per_cu == 0) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kern),
                                                     kPairThreads, bytes) != hipSuccess || n < 1)
      n = 1;
    per_cu = n;
  }
  const int ntiles = LB.B * ((LB.H + kPairTH - 1) / kPairTH) * ((LB.W + kPairTW - 1) / kPairTW);
  const int nb = ntiles < per_cu * cu_count() ? ntiles : per_cu * cu_count();
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kPairThreads), bytes, s, LA, LB, ntiles);
}

bool launch_conv_pair(const ConvArgs& LA, int in_mode, const ConvArgs& LB, int out_mode,
                      hipStream_t s) {
  // Only the first pair (state -> 48 -> 48) has a fused kernel: its layer A is small (K = 27)
  // and its weights small, so 16-row tiles (16 waves) fit.  Two 48-channel layers need both
  // weight sets in LDS (83 KB), which leaves room for 8-row tiles only (10 waves, layer A on
  // 1.33x the cells); measured, such pairs were slower than two one-layer passes.
  if (LA.cout != 48 || LA.Npad != 48 || LB.cin != 48 || LB.Kpad != TileGeom<48>::KP) return false;
  if (in_mode == kInStateNorm && LA.cin == 3 && LA.Kpad == 32 && LB.cout == 48 &&
      LB.Npad == 48 && out_mode == kOutReluBf16) {
    launch_pair_t<8, kInStateNorm, 3, kOutReluBf16, 14>(LA, LB, s);
    return true;
  }
  return false;
}

void launch_wgrad(const ConvArgs& A, int in_mode, const uint16_t* g, int gch, int cells_per_chunk,
                  float* part, hipStream_t s) {
  const int ncells = A.B * A.H * A.W;
  const int nchunks = (ncells + cells_per_chunk - 1) / cells_per_chunk;
  const int waves = nchunks * (A.Kpad / 16);
  if (in_mode == kInStateNorm)
    hipLaunchKernelGGL(wgrad_mfma_kernel<kInStateNorm>, dim3((waves + 3) / 4), dim3(256), 0, s, A, g,
                       gch, cells_per_chunk, part, waves);
  else
    hipLaunchKernelGGL(wgrad_mfma_kernel<kInNhwcVec>, dim3((waves + 3) / 4), dim3(256), 0, s, A, g,
                       gch, cells_per_chunk, part, waves);
}

void launch_bgrad(const uint16_t* g, int gch, int ncells, int cells_per_chunk, float* part,
                  hipStream_t s) {
  const int nchunks = (ncells + cells_per_chunk - 1) / cells_per_chunk;
  hipLaunchKernelGGL(bgrad_kernel, dim3(nchunks), dim3(64), 0, s, g, gch, ncells, cells_per_chunk,
                     part);
}

void launch_reduce_grads(const float* wpart, const float* bpart, int nchunks, int cin, int cout,
                         int Kpad, int Npad, float* gw, float* gb, hipStream_t s) {
  const int n = cout * cin * 9 + cout;
  hipLaunchKernelGGL(reduce_grads_kernel, dim3((n + 255) / 256), dim3(256), 0, s, wpart, bpart,
                     nchunks, cin, cout, Kpad, Npad, gw, gb);
}

void launch_mse(const float* y, const float* st_in, const float* st_tgt, int B, int H, int W,
                const float sc[3], uint16_t* g, float* lpart, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, s, y, st_in, st_tgt, B, H, W, sc[0],
                     sc[1], sc[2], g, lpart);
}

void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
}

void launch_prep_weights(const float* w, int cin, int cout, int Kf, int Npf, int Kd, int Npd,
                         uint16_t* wf, uint16_t* wd, hipStream_t s) {
  const int n = Npf * Kf + (wd ? Npd * Kd : 0);
  hipLaunchKernelGGL(prep_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, cin, cout, Kf,
                     Npf, Kd, Npd, wf, wd);
}

int channel_stats_parts() { return 3 * kStatBlocks * 4; }

void launch_channel_stats(const float* x, const float* t, int B, int hw, double* part, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(channel_moments_kernel, dim3(kStatBlocks, 3), dim3(256), 0, s, x, t, B, hw,
                     part);
  hipLaunchKernelGGL(channel_moments_finish_kernel, dim3(1), dim3(64), 0, s, part,
                     (double)B * hw, out);
}

void launch_count_flags(const int32_t* flags, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(count_flags_kernel, dim3(1), dim3(64), 0, s, flags, n, out);
}

void launch_copy_flagged(const float* src, float* dst, const int32_t* flags, int ne, size_t per,
                         hipStream_t s) {
  size_t bx = (per + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(copy_flagged_kernel, dim3((unsigned)bx, ne), dim3(256), 0, s, src, dst, flags,
                     per);
}

void launch_mass_drift(const float* before, const float* after, int ne, int ncell, double H,
                       double tol, double* drift, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(mass_drift_kernel, dim3(ne), dim3(256), 0, s, before, after, ncell, H, tol,
                     drift, flags);
}

}  // namespace iewpf
