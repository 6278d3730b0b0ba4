// Covariance-operator kernels: normals on the coarse random grid, the SOAR stencil, and the
// fine-grid pass Q_GB^{1/2} I_Omega (bicubic + geostrophic balance) that adds a coarse field
// into the state, optionally together with the optimal-proposal pull windows.
//
// Paper: Section "Small scale model errors" (eq. soar_function, eq. local_soar_on_eta,
// eq. geostrophic_balance_disc), Section "Efficient generation of model errors" (one
// output element per work-item, perturbation never stored), Section "Optimal proposal
// particles" (pull chain, eq. detailedOPDUpdate) and "Posterior particle states"
// (eq. optUpdateEquationTwoStage).
#include "buffer_dev.hpp"
#include "internal.hpp"
#include "philox_dev.hpp"

namespace iewpf {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}
// i in [-n, 2n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ __forceinline__ int floordiv(int a, int b) {  // b > 0
  const int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Catmull-Rom weights (taps -1, 0, 1, 2) at phase p in [0, 2c) of a fine row or column,
// t = p / (2c).
__device__ __forceinline__ void cr_phase(const CoarseConst& C, int p, float w[4]) {
  const float t = static_cast<float>(p) * (1.0f / static_cast<float>(2 * C.c));
  const float t2 = t * t, t3 = t2 * t;
  w[0] = 0.5f * (-t3 + 2.0f * t2 - t);
  w[1] = 0.5f * (3.0f * t3 - 5.0f * t2 + 2.0f);
  w[2] = 0.5f * (-3.0f * t3 + 4.0f * t2 + t);
  w[3] = 0.5f * (t3 - t2);
}

// x-interpolated coarse rows around the current fine row (see swe_kernels.hip for the
// same scheme): the window advances one coarse row every c fine rows.
struct CoarseWin {
  float xr[4];
  int by;
  __device__ __forceinline__ float xrow(const float* __restrict__ z, const CoarseConst& C,
                                        const int cx[4], const float wx[4], int b) const {
    const float* row = z + (size_t)wrap1(b, C.nry) * C.nrx;
    return wx[0] * row[cx[0]] + wx[1] * row[cx[1]] + wx[2] * row[cx[2]] + wx[3] * row[cx[3]];
  }
  __device__ __forceinline__ void init(const float* __restrict__ z, const CoarseConst& C,
                                       const int cx[4], const float wx[4], int s) {
    by = floordiv(2 * s + 1 - C.c, 2 * C.c);
#pragma unroll
    for (int n = 0; n < 4; ++n) xr[n] = xrow(z, C, cx, wx, by + n - 1);
  }
  // fine row s (unwrapped), called with s increasing by one
  __device__ __forceinline__ float at(const float* __restrict__ z, const CoarseConst& C,
                                      const int cx[4], const float wx[4], int s) {
    const int num = 2 * s + 1 - C.c;
    const int b = floordiv(num, 2 * C.c);
    if (b != by) {
      xr[0] = xr[1];
      xr[1] = xr[2];
      xr[2] = xr[3];
      xr[3] = xrow(z, C, cx, wx, b + 2);
      by = b;
    }
    float wy[4];
    cr_phase(C, num - 2 * C.c * b, wy);
    return wy[0] * xr[0] + wy[1] * xr[1] + wy[2] * xr[2] + wy[3] * xr[3];
  }
};

struct Stencil25 {
  float w[25];
};

// step index = step + dyn[0] when dyn is set (counters read from device memory so that a
// captured graph advances its streams between replays)
__global__ __launch_bounds__(256) void normals_kernel(float* __restrict__ out, int n, uint64_t seed,
                                                      uint64_t step, uint32_t tag, uint32_t ens,
                                                      const uint64_t* __restrict__ dyn) {
  const int blk = blockIdx.x * blockDim.x + threadIdx.x;
  const int particle = blockIdx.y;
  if (4 * blk >= n) return;
  double z[4];
  normals4(blk, step + blockIdx.z + (dyn ? dyn[0] : 0), tag, ens, particle, seed, z);
  float* o = out + ((size_t)blockIdx.z * gridDim.y + particle) * n;
#pragma unroll
  for (int l = 0; l < 4; ++l)
    if (4 * blk + l < n) o[4 * blk + l] = static_cast<float>(z[l]);
}

__global__ __launch_bounds__(256) void soar_kernel(const float* __restrict__ in,
                                                   float* __restrict__ out, int nrx, int nry,
                                                   Stencil25 W) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = nrx * nry;
  if (p >= nr) return;
  const int particle = blockIdx.y;
  const int b = p / nrx, a = p - b * nrx;
  const float* src = in + (size_t)particle * nr;
  float acc = 0.0f;
#pragma unroll
  for (int q = -2; q <= 2; ++q) {
    const float* row = src + (size_t)wrap1(b + q, nry) * nrx;
#pragma unroll
    for (int pp = -2; pp <= 2; ++pp) acc += W.w[(q + 2) * 5 + (pp + 2)] * row[wrap1(a + pp, nrx)];
  }
  out[(size_t)particle * nr + p] = acc;
}

// Bicubic value of the coarse field z (one particle) at fine cell (j, k) given the lane's
// x taps.
__device__ __forceinline__ float bicubic_at(const float* __restrict__ z, const CoarseConst& C,
                                            const int cx[4], const float wx[4], int k) {
  const int num = 2 * k + 1 - C.c;
  const int by = floordiv(num, 2 * C.c);
  float wy[4];
  cr_phase(C, num - 2 * C.c * by, wy);
  float acc = 0.0f;
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const float* row = z + (size_t)wrap1(by + n - 1, C.nry) * C.nrx;
    const float rv = wx[0] * row[cx[0]] + wx[1] * row[cx[1]] + wx[2] * row[cx[2]] + wx[3] * row[cx[3]];
    acc += wy[n] * rv;
  }
  return acc;
}

// Fine pass over wave strips of 62 output columns (lanes 1..62) marching down rows:
//   psi(k) = (base or psi)(k) + (d_eta, -gH/(2 f dy) (d_eta(k+1) - d_eta(k-1)),
//                                 gH/(2 f dx) (d_eta(j+1) - d_eta(j-1)))  [+ pull windows]
// with d_eta = I_Omega z.
__global__ __launch_bounds__(256) void gb_add_kernel(CoarseConst C, int strip_h, int n_strip_x,
                                                     int n_strip_y, int total_waves,
                                                     const float* __restrict__ zall,
                                                     const float* __restrict__ base,
                                                     float* __restrict__ psi) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wave >= total_waves) return;
  const int per_particle = n_strip_x * n_strip_y;
  const int particle = wave / per_particle;
  const int strip = wave - particle * per_particle;
  const int sy = strip / n_strip_x;
  const int sx = strip - sy * n_strip_x;
  const int nx = C.nx, ny = C.ny;
  const size_t ncell = (size_t)nx * ny;
  const float* z = zall + (size_t)particle * C.nrx * C.nry;
  float* E = psi + (size_t)particle * 3 * ncell;
  const float* B = base ? base : E;  // base: one shared state [3][ny][nx]

  const int j = sx * kGbOut + lane - kGbHalo;
  const int jw = wrapi(j, nx);
  const bool writer = lane >= kGbHalo && lane < kWave - kGbHalo && j < nx;
  // x taps of this lane (unshifted coarse grid: coarse point a at (a + 1/2) c dx)
  int cx[4];
  float wx[4];
  {
    const int num = 2 * jw + 1 - C.c;
    const int bx = floordiv(num, 2 * C.c);
    cr_phase(C, num - 2 * C.c * bx, wx);
#pragma unroll
    for (int m = 0; m < 4; ++m) cx[m] = wrap1(bx + m - 1, C.nrx);
  }
  const int k0 = sy * strip_h;
  const int k_end = min(k0 + strip_h, ny);
  float dm2 = 0.0f, dm1 = 0.0f;  // d_eta rows m-2, m-1
  CoarseWin win;
  win.init(z, C, cx, wx, k0 - 1);
  for (int m = k0 - 1; m <= k_end; ++m) {
    const float d0 = win.at(z, C, cx, wx, m);
    if (m >= k0 + 1) {
      const int k = m - 1;
      const float de = dm1;
      const float dhu = -C.gb_y * (d0 - dm2);
      const float dhv = C.gb_x * (__shfl_down(dm1, 1, kWave) - __shfl_up(dm1, 1, kWave));
      if (writer) {
        const size_t o = (size_t)k * nx + j;
        E[o] = B[o] + de;
        E[ncell + o] = B[ncell + o] + dhu;
        E[2 * ncell + o] = B[2 * ncell + o] + dhv;
      }
    }
    dm2 = dm1;
    dm1 = d0;
  }
}

// Analysis update, one fused pass over the state (eq. optUpdateEquationTwoStage with the
// pull of eq. detailedOPDUpdate): psi += sum_o (s_u,o W_u + s_v,o W_v)(x - x_o) + Q_GB I_Omega z
// for kPB particles per wave, so every window value fetched from cache serves kPB
// particles.  W_u, W_v: precomputed responses to the unit vectors (stored windows); the
// observation list of the strip comes from the host with each window's origin on the torus,
// and S d in float32, both read with scalar loads; the row window test is wave-uniform.
constexpr int kPB = kUpdParticles;
#ifndef IEWPF_UPD_OBS_BATCH
#define IEWPF_UPD_OBS_BATCH 4
#endif
constexpr int kObsBatch = IEWPF_UPD_OBS_BATCH;


// SIMPLE_X: the grid is at least a window plus a wave wide and the windows are not folded,
// so a strip's lanes meet each window at most once and every entry carries the byte offset
// of lane 0's window column (negative when the window starts to the left of the strip);
// otherwise the entry carries the window's first column and every lane wraps its own offset.
// WS: the window row stride per field in floats (0: runtime, P.ws).
template <bool SIMPLE_X, int WS>
__global__ __launch_bounds__(256, 5) void analysis_update_kernel(
    CoarseConst C, PullConst P, int ne, int ne4, int total_waves, const float* __restrict__ zall,
    float* __restrict__ psi, const float* __restrict__ windows, const float* __restrict__ sdf,
    const int2* __restrict__ st_rows, const int4* __restrict__ st_ent,
    double* __restrict__ scal, int32_t* __restrict__ host_flag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave));
  if (wave >= total_waves) return;
  int32_t* status = reinterpret_cast<int32_t*>(scal + kScalStatus);
  if (status[0] & kStatSkipUpdate) return;  // beta <= 0 or non-finite scalars: state untouched
  const int per_group = P.n_strip_x * P.n_strip_y;
  const int group = wave / per_group;
  const int strip = wave - group * per_group;
  const int sy = strip / P.n_strip_x;
  const int sx = strip - sy * P.n_strip_x;
  const int p0 = group * kPB;
  const int np = min(kPB, ne - p0);
  const int nx = C.nx, ny = C.ny;
  const size_t ncell = (size_t)nx * ny;
  const unsigned ws4 = 4u * static_cast<unsigned>(WS > 0 ? WS : P.ws);  // field stride, bytes
  const unsigned wrow4 = 6u * ws4;                                       // window row, bytes
  const unsigned wx4 = 4u * static_cast<unsigned>(P.wx);

  const int j = sx * kGbOut + lane - kGbHalo;
  const int jw = wrapi(j, nx);
  const unsigned lane4 = 4u * static_cast<unsigned>(lane);
  const bool writer = lane >= kGbHalo && lane < kWave - kGbHalo && j < nx;
  // State and windows as raw buffers (byte offsets < 2^31, checked when the context is
  // created): state rows by a scalar offset and one lane offset, which switches the lanes
  // that write nothing off (reads zero, writes dropped); a group's missing particles get
  // an empty buffer.
  const unsigned bj = writer ? 4u * static_cast<unsigned>(j) : kBufferOff;
  const unsigned brow = 4u * static_cast<unsigned>(nx);
  const unsigned fq = 4u * static_cast<unsigned>(ncell), fr = 2u * fq;
  __amdgpu_buffer_rsrc_t bs[kPB];
#pragma unroll
  for (int p = 0; p < kPB; ++p)
    bs[p] = make_rsrc(psi + (size_t)min(p0 + p, ne - 1) * 3 * ncell, p < np ? 12 * ncell : 0);
  const __amdgpu_buffer_rsrc_t bw = make_rsrc(windows, (size_t)P.wy * wrow4);
  const char* sdf_g = reinterpret_cast<const char*>(sdf + 2 * (size_t)p0);
  int cx[4];
  float wx[4];
  {
    const int num = 2 * jw + 1 - C.c;
    const int bx = floordiv(num, 2 * C.c);
    cr_phase(C, num - 2 * C.c * bx, wx);
#pragma unroll
    for (int m = 0; m < 4; ++m) cx[m] = wrap1(bx + m - 1, C.nrx);
  }
  const int k0 = sy * P.strip_h;
  const int k_end = min(k0 + P.strip_h, ny);
  // Per row, the range of list entries whose windows hold the row (entry 0: a sentinel whose
  // S d row is zero, which pads the last batch): per entry the window's column (see SIMPLE_X),
  // its first row on the torus (the observed cell minus the radius; the cell itself for a
  // window folded onto the whole period) and the byte offset of the observation's S d row;
  // read with scalar loads (the index is wave-uniform), as are S d of the group's particles
  // (float, observation-major).
  const int2* rows = st_rows + (size_t)sx * ny;
  float dm2[kPB], dm1[kPB];
  float chk[kPB];  // stays 0 while every written value is finite (x * 0 is NaN for inf, NaN)
  CoarseWin win[kPB];
#pragma unroll
  for (int p = 0; p < kPB; ++p) {
    chk[p] = 0.0f;
    dm2[p] = dm1[p] = 0.0f;
    win[p].init(zall + (size_t)min(p0 + p, ne - 1) * C.nrx * C.nry, C, cx, wx, k0 - 1);
  }
  for (int m = k0 - 1; m <= k_end; ++m) {
    float d0[kPB];
#pragma unroll
    for (int p = 0; p < kPB; ++p)
      d0[p] = win[p].at(zall + (size_t)min(p0 + p, ne - 1) * C.nrx * C.nry, C, cx, wx, m);
    if (m >= k0 + 1) {
      const int k = m - 1;
      float ae[kPB], au[kPB], av[kPB];
      float se[kPB], su_[kPB], sv_[kPB];  // state values, loaded before the observation loop
      const unsigned srow = static_cast<unsigned>(k) * brow;
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        se[p] = ld_buf(bs[p], bj, srow);
        su_[p] = ld_buf(bs[p], bj, srow + fq);
        sv_[p] = ld_buf(bs[p], bj, srow + fr);
      }
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        ae[p] = dm1[p];
        au[p] = -C.gb_y * (d0[p] - dm2[p]);
        av[p] = C.gb_x * (__shfl_down(dm1[p], 1, kWave) - __shfl_up(dm1[p], 1, kWave));
      }
      // kObsBatch observations at a time: all window loads of a batch issued before its
      // multiply-adds
      const int2 range = rows[k];
      const int o_beg = range.x, o_end = range.y;
      for (int t0 = o_beg; t0 < o_end; t0 += kObsBatch) {
        float w[kObsBatch][6];
        float su[kObsBatch][kPB], sv[kObsBatch][kPB];
#pragma unroll
        for (int u = 0; u < kObsBatch; ++u) {
          const int4 e = st_ent[t0 + u < o_end ? t0 + u : 0];  // wave-uniform
          int iy = k - e.y;  // 0 <= k, e.y < ny: the window row on the torus
          iy += iy < 0 ? ny : 0;
          const unsigned soff = static_cast<unsigned>(iy) * wrow4;
          unsigned voff;
          if (SIMPLE_X) {
            const unsigned v = lane4 + static_cast<unsigned>(e.x);
            voff = v < wx4 ? v : kBufferOff;
          } else {
            int ix = jw - e.x;  // 0 <= jw, e.x < nx
            ix += ix < 0 ? nx : 0;
            voff = static_cast<unsigned>(ix) < static_cast<unsigned>(P.wx)
                       ? 4u * static_cast<unsigned>(ix)
                       : kBufferOff;
          }
#pragma unroll
          for (int f = 0; f < 6; ++f) w[u][f] = ld_buf(bw, voff + f * ws4, soff);
          const float* q = reinterpret_cast<const float*>(sdf_g + static_cast<unsigned>(e.z));
#pragma unroll
          for (int p = 0; p < kPB; ++p) {
            su[u][p] = q[2 * p];
            sv[u][p] = q[2 * p + 1];
          }
        }
#pragma unroll
        for (int u = 0; u < kObsBatch; ++u) {
#pragma unroll
          for (int p = 0; p < kPB; ++p) {
            ae[p] = fmaf(sv[u][p], w[u][3], fmaf(su[u][p], w[u][0], ae[p]));
            au[p] = fmaf(sv[u][p], w[u][4], fmaf(su[u][p], w[u][1], au[p]));
            av[p] = fmaf(sv[u][p], w[u][5], fmaf(su[u][p], w[u][2], av[p]));
          }
        }
      }
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        const float oe = se[p] + ae[p], ou = su_[p] + au[p], ov = sv_[p] + av[p];
        st_buf(bs[p], bj, srow, oe);
        st_buf(bs[p], bj, srow + fq, ou);
        st_buf(bs[p], bj, srow + fr, ov);
        chk[p] = fmaf(ov, 0.0f, fmaf(ou, 0.0f, fmaf(oe, 0.0f, chk[p])));
      }
    }
#pragma unroll
    for (int p = 0; p < kPB; ++p) {
      dm2[p] = dm1[p];
      dm1[p] = d0[p];
    }
  }
  // a particle with a non-finite written value: flag it (rare; the atomic minimum gives the
  // same particle whatever the order of the waves)
#pragma unroll
  for (int p = 0; p < kPB; ++p) {
    const bool bad = writer && p < np && !isfinite(chk[p]);
    if (__ballot(bad) != 0 && lane == 0) {
      atomicOr(status + 2, kStatNonfiniteState);
      atomicMin(status + 3, p0 + p);
      if (host_flag) *host_flag = 1;  // the host then reads the device status words
    }
  }
}

// The same update with the pull windows staged in LDS once per workgroup, cell-major
// ([wy * wx + 1][6], the last cell zero: the lanes a window misses read it).  Window reads then
// wait only on the LDS counter, so the state rows can be loaded one row ahead and the coarse
// rows of the random part one fine row ahead without the observation loop waiting on them;
// the arithmetic is that of analysis_update_kernel, in the same order.
#ifndef IEWPF_UPD_LDS_WAVES
#define IEWPF_UPD_LDS_WAVES 8
#endif
#ifndef IEWPF_UPD_LDS_OCC
#define IEWPF_UPD_LDS_OCC 4
#endif
constexpr int kLdsWaves = IEWPF_UPD_LDS_WAVES;
#ifndef IEWPF_UPD_DEPTH
#define IEWPF_UPD_DEPTH 1
#endif
constexpr int kUpdDepth = IEWPF_UPD_DEPTH;  // state rows loaded ahead

template <bool SIMPLE_X>
__global__ __launch_bounds__(kLdsWaves * kWave, IEWPF_UPD_LDS_OCC) void analysis_update_lds_kernel(
    CoarseConst C, PullConst P, int ne, int ne4, int total_waves, const float* __restrict__ zall,
    float* __restrict__ psi, const float* __restrict__ wcell, const float* __restrict__ sdf,
    const int2* __restrict__ st_rows, const int4* __restrict__ st_ent,
    double* __restrict__ scal, int32_t* __restrict__ host_flag) {
  extern __shared__ __align__(16) float lw[];
  int32_t* status = reinterpret_cast<int32_t*>(scal + kScalStatus);
  if (status[0] & kStatSkipUpdate) return;  // the same for every workgroup
  const int ncw = P.wx * P.wy;
  {
    // stage the windows (padded to whole 1 KB chunks) with LDS-direct loads: each lane of a
    // wave moves 16 bytes of a chunk straight into LDS, lane l to byte 16 l of the chunk
    const int n4 = update_lds_float4s(P.wx, P.wy);
    const float4* src = reinterpret_cast<const float4*>(wcell) + (threadIdx.x & (kWave - 1));
    for (int ch = threadIdx.x / kWave; ch * kWave < n4; ch += kLdsWaves)
      __builtin_amdgcn_global_load_lds(
          (__attribute__((address_space(1))) void*)(const_cast<float4*>(src + ch * kWave)),
          (__attribute__((address_space(3))) void*)(lw + ch * 4 * kWave), 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * kLdsWaves + (threadIdx.x / kWave));
  if (wave >= total_waves) return;
  const int per_group = P.n_strip_x * P.n_strip_y;
  const int group = wave / per_group;
  const int strip = wave - group * per_group;
  const int sy = strip / P.n_strip_x;
  const int sx = strip - sy * P.n_strip_x;
  const int p0 = group * kPB;
  const int np = min(kPB, ne - p0);
  const int nx = C.nx, ny = C.ny;
  const size_t ncell = (size_t)nx * ny;
  const int nrc = C.nrx * C.nry;

  const int j = sx * kGbOut + lane - kGbHalo;
  const int jw = wrapi(j, nx);
  const bool writer = lane >= kGbHalo && lane < kWave - kGbHalo && j < nx;
  const unsigned bj = writer ? 4u * static_cast<unsigned>(j) : kBufferOff;
  const unsigned brow = 4u * static_cast<unsigned>(nx);
  const unsigned fq = 4u * static_cast<unsigned>(ncell), fr = 2u * fq;
  __amdgpu_buffer_rsrc_t bs[kPB], bz[kPB];
#pragma unroll
  for (int p = 0; p < kPB; ++p) {
    const int q = min(p0 + p, ne - 1);
    bs[p] = make_rsrc(psi + (size_t)q * 3 * ncell, p < np ? 12 * ncell : 0);
    bz[p] = make_rsrc(zall + (size_t)q * nrc, 4 * (size_t)nrc);
  }
  const char* sdf_g = reinterpret_cast<const char*>(sdf + 2 * (size_t)p0);
  const unsigned lane24 = 24u * static_cast<unsigned>(lane);
  const unsigned wx24 = 24u * static_cast<unsigned>(P.wx);
  const unsigned zero24 = 24u * static_cast<unsigned>(ncw);
  int cx[4];
  float wxw[4];
  unsigned cxo[4];  // byte offsets of the lane's coarse columns
  {
    const int num = 2 * jw + 1 - C.c;
    const int bx = floordiv(num, 2 * C.c);
    cr_phase(C, num - 2 * C.c * bx, wxw);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cx[m] = wrap1(bx + m - 1, C.nrx);
      cxo[m] = 4u * static_cast<unsigned>(cx[m]);
    }
  }
  const unsigned crow = 4u * static_cast<unsigned>(C.nrx);
  auto coarse_row = [&](int b) { return static_cast<unsigned>(wrap1(b, C.nry)) * crow; };
  auto brow_of = [&](int s) { return floordiv(2 * s + 1 - C.c, 2 * C.c); };
  const int k0 = sy * P.strip_h;
  const int k_end = min(k0 + P.strip_h, ny);
  const int2* rows = st_rows + (size_t)sx * ny;

  // x-interpolated coarse rows by-1 .. by+2 around fine row s (as CoarseWin) and the raw taps
  // of row by+3, loaded as soon as the previous row moved in (a coarse period ahead)
  float xr[kPB][4];
  float pre[kPB][4];
  int by = brow_of(k0 - 1);
#pragma unroll
  for (int p = 0; p < kPB; ++p)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const unsigned ro = coarse_row(by + n - 1);
      float v[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) v[a] = ld_buf(bz[p], cxo[a], ro);
      xr[p][n] = wxw[0] * v[0] + wxw[1] * v[1] + wxw[2] * v[2] + wxw[3] * v[3];
    }
  auto load_next_coarse = [&]() {
    const unsigned ro = coarse_row(by + 3);
#pragma unroll
    for (int p = 0; p < kPB; ++p)
#pragma unroll
      for (int a = 0; a < 4; ++a) pre[p][a] = ld_buf(bz[p], cxo[a], ro);
  };
  load_next_coarse();
  // d at fine row s (s increasing by one per call)
  auto d_at = [&](int s, float (&d)[kPB]) {
    const int num = 2 * s + 1 - C.c;
    const int b = floordiv(num, 2 * C.c);
    if (b != by) {
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        xr[p][0] = xr[p][1];
        xr[p][1] = xr[p][2];
        xr[p][2] = xr[p][3];
        xr[p][3] = wxw[0] * pre[p][0] + wxw[1] * pre[p][1] + wxw[2] * pre[p][2] + wxw[3] * pre[p][3];
      }
      by = b;
      load_next_coarse();
    }
    float wy[4];
    cr_phase(C, num - 2 * C.c * b, wy);
#pragma unroll
    for (int p = 0; p < kPB; ++p)
      d[p] = wy[0] * xr[p][0] + wy[1] * xr[p][1] + wy[2] * xr[p][2] + wy[3] * xr[p][3];
  };
  float dm2[kPB], dm1[kPB];
  float chk[kPB];
#pragma unroll
  for (int p = 0; p < kPB; ++p) chk[p] = 0.0f;
  d_at(k0 - 1, dm2);
  d_at(k0, dm1);
  // state rows kUpdDepth rows ahead in a ring of kUpdDepth + 1 rows
  float st[kUpdDepth + 1][3][kPB];
  auto load_row = [&](int k, float (&sr)[3][kPB]) {
    const unsigned srow = static_cast<unsigned>(k) * brow;
#pragma unroll
    for (int p = 0; p < kPB; ++p) {
      sr[0][p] = ld_buf(bs[p], bj, srow);
      sr[1][p] = ld_buf(bs[p], bj, srow + fq);
      sr[2][p] = ld_buf(bs[p], bj, srow + fr);
    }
  };
#pragma unroll
  for (int u = 0; u < kUpdDepth; ++u)
    if (k0 + u < k_end) load_row(k0 + u, st[u]);
  // output row k from state row k (cur); issues the loads of row k + kUpdDepth (ahead) first
  auto body = [&](int k, float (&cur)[3][kPB], float (&ahead)[3][kPB]) {
    if (k + kUpdDepth < k_end) load_row(k + kUpdDepth, ahead);
    float d0[kPB];
    d_at(k + 1, d0);
    float ae[kPB], au[kPB], av[kPB];
#pragma unroll
    for (int p = 0; p < kPB; ++p) {
      ae[p] = dm1[p];
      au[p] = -C.gb_y * (d0[p] - dm2[p]);
      av[p] = C.gb_x * (__shfl_down(dm1[p], 1, kWave) - __shfl_up(dm1[p], 1, kWave));
    }
    const int2 range = rows[k];
    const int o_beg = range.x, o_end = range.y;
    for (int t0 = o_beg; t0 < o_end; t0 += kObsBatch) {
      float w[kObsBatch][6];
      float su[kObsBatch][kPB], sv[kObsBatch][kPB];
#pragma unroll
      for (int u = 0; u < kObsBatch; ++u) {
        const int4 e = st_ent[t0 + u < o_end ? t0 + u : 0];  // wave-uniform
        int iy = k - e.y;
        iy += iy < 0 ? ny : 0;
        const unsigned rbase = static_cast<unsigned>(iy) * wx24;
        unsigned off;
        if (SIMPLE_X) {
          const unsigned v = lane24 + static_cast<unsigned>(e.w);
          off = v < wx24 ? rbase + v : zero24;
        } else {
          int ix = jw - e.x;
          ix += ix < 0 ? nx : 0;
          off = ix < P.wx ? rbase + 24u * static_cast<unsigned>(ix) : zero24;
        }
        const float2* c2 = reinterpret_cast<const float2*>(reinterpret_cast<const char*>(lw) + off);
        const float2 w01 = c2[0], w23 = c2[1], w45 = c2[2];
        w[u][0] = w01.x;
        w[u][1] = w01.y;
        w[u][2] = w23.x;
        w[u][3] = w23.y;
        w[u][4] = w45.x;
        w[u][5] = w45.y;
        const float* q = reinterpret_cast<const float*>(sdf_g + static_cast<unsigned>(e.z));
#pragma unroll
        for (int p = 0; p < kPB; ++p) {
          su[u][p] = q[2 * p];
          sv[u][p] = q[2 * p + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < kObsBatch; ++u) {
#pragma unroll
        for (int p = 0; p < kPB; ++p) {
          ae[p] = fmaf(sv[u][p], w[u][3], fmaf(su[u][p], w[u][0], ae[p]));
          au[p] = fmaf(sv[u][p], w[u][4], fmaf(su[u][p], w[u][1], au[p]));
          av[p] = fmaf(sv[u][p], w[u][5], fmaf(su[u][p], w[u][2], av[p]));
        }
      }
    }
    const unsigned srow = static_cast<unsigned>(k) * brow;
#pragma unroll
    for (int p = 0; p < kPB; ++p) {
      const float oe = cur[0][p] + ae[p], ou = cur[1][p] + au[p], ov = cur[2][p] + av[p];
      st_buf(bs[p], bj, srow, oe);
      st_buf(bs[p], bj, srow + fq, ou);
      st_buf(bs[p], bj, srow + fr, ov);
      chk[p] = fmaf(ov, 0.0f, fmaf(ou, 0.0f, fmaf(oe, 0.0f, chk[p])));
      dm2[p] = dm1[p];
      dm1[p] = d0[p];
    }
  };
  for (int kb = k0; kb < k_end; kb += kUpdDepth + 1) {
#pragma unroll
    for (int u = 0; u <= kUpdDepth; ++u)
      if (kb + u < k_end) body(kb + u, st[u], st[(u + kUpdDepth) % (kUpdDepth + 1)]);
  }
#pragma unroll
  for (int p = 0; p < kPB; ++p) {
    const bool bad = writer && p < np && !isfinite(chk[p]);
    if (__ballot(bad) != 0 && lane == 0) {
      atomicOr(status + 2, kStatNonfiniteState);
      atomicMin(status + 3, p0 + p);
      if (host_flag) *host_flag = 1;  // the host then reads the device status words
    }
  }
}

}  // namespace

void launch_normals(float* out, int n, int ne, uint64_t seed, uint64_t step, uint32_t tag,
                    uint32_t ens, hipStream_t s, const uint64_t* dyn, int n_steps) {
  const int nblk = (n + 3) / 4;
  hipLaunchKernelGGL(normals_kernel, dim3((nblk + 255) / 256, ne, n_steps), dim3(256), 0, s, out, n,
                     seed, step, tag, ens, dyn);
}

void launch_soar(const CoarseConst& C, const float* w25, int ne, const float* in, float* out,
                 hipStream_t s) {
  Stencil25 W;
  for (int i = 0; i < 25; ++i) W.w[i] = w25[i];
  const int nr = C.nrx * C.nry;
  hipLaunchKernelGGL(soar_kernel, dim3((nr + 255) / 256, ne), dim3(256), 0, s, in, out, C.nrx,
                     C.nry, W);
}

void launch_gb_add(const CoarseConst& C, int ne, const float* z, const float* base, float* psi,
                   int strip_h, hipStream_t s) {
  const int nsx = (C.nx + kGbOut - 1) / kGbOut;
  const int nsy = (C.ny + strip_h - 1) / strip_h;
  const int total = ne * nsx * nsy;
  hipLaunchKernelGGL(gb_add_kernel, dim3((total + 3) / 4), dim3(256), 0, s, C, strip_h, nsx, nsy,
                     total, z, base, psi);
}

int update_waves_per_cu() {
  int a = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, analysis_update_kernel<true, kWinStride>,
                                                   256, 0) != hipSuccess)
    return 16;
  return 4 * (a > 0 ? a : 1);
}

int update_particle_group() { return kPB; }

size_t update_lds_bytes(int wx, int wy) { return 16 * (size_t)update_lds_float4s(wx, wy); }

int update_lds_waves_per_cu() {
  int a = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, analysis_update_lds_kernel<true>,
                                                   kLdsWaves * kWave, 0) != hipSuccess)
    return 16;
  return kLdsWaves * (a > 0 ? a : 1);
}

void launch_analysis_update(const CoarseConst& C, const PullConst& P, int ne, const float* z,
                            const float* windows, const float* wcell, const float* sdf,
                            const int32_t* st_rows, const int32_t* st_ent, float* psi,
                            double* scal, int32_t* host_flag, hipStream_t s) {
  const int groups = (ne + kPB - 1) / kPB;
  const int total = groups * P.n_strip_x * P.n_strip_y;
  const int2* rows = reinterpret_cast<const int2*>(st_rows);
  const int4* ent = reinterpret_cast<const int4*>(st_ent);
  const int ne4 = sd_float_stride(ne);
  if (wcell) {
    const size_t lds = update_lds_bytes(P.wx, P.wy);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(analysis_update_lds_kernel<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kUpdateLdsMax);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(analysis_update_lds_kernel<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kUpdateLdsMax);
      attr = true;
    }
    const dim3 grid((total + kLdsWaves - 1) / kLdsWaves), block(kLdsWaves * kWave);
    if (P.simple_x)
      hipLaunchKernelGGL((analysis_update_lds_kernel<true>), grid, block, lds, s, C, P, ne, ne4,
                         total, z, psi, wcell, sdf, rows, ent, scal, host_flag);
    else
      hipLaunchKernelGGL((analysis_update_lds_kernel<false>), grid, block, lds, s, C, P, ne, ne4,
                         total, z, psi, wcell, sdf, rows, ent, scal, host_flag);
    return;
  }
  const dim3 grid((total + 3) / 4), block(256);
  const bool fixed = P.ws == kWinStride;
  if (P.simple_x && fixed)
    hipLaunchKernelGGL((analysis_update_kernel<true, kWinStride>), grid, block, 0, s, C, P, ne, ne4,
                       total, z, psi, windows, sdf, rows, ent, scal, host_flag);
  else if (fixed)
    hipLaunchKernelGGL((analysis_update_kernel<false, kWinStride>), grid, block, 0, s, C, P, ne,
                       ne4, total, z, psi, windows, sdf, rows, ent, scal, host_flag);
  else
    hipLaunchKernelGGL((analysis_update_kernel<false, 0>), grid, block, 0, s, C, P, ne, ne4, total,
                       z, psi, windows, sdf, rows, ent, scal, host_flag);
}

}  // namespace iewpf
