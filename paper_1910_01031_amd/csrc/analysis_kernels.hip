// IEWPF analysis kernels (Section "Efficient implementation of the IEWPF scheme",
// Appendix A) plus observation synthesis, the CFL check, drifters and residual resampling.
//
//   innovation_kernel     stage 1-2: d = y (H + eta)/H - (hu, hv) (eq. etaCompensatedInnovation),
//                         S d, c_i = sum_o d^T S d (eq. ciMultiDrifter), float64
//   rand_dots_kernel      stage 3: xi, nu~ ~ N(0, I) on Omega^R and xi.xi, nu~.nu~, nu~.xi
//   sync_kernel           stages 4-5, the only ensemble-wide step: cbar, beta
//                         (eq. betaTwoStage), c*_i (eq. cistarTwoStage), alpha_i by the
//                         principal Lambert W branch (eq. iewpfAlphaSol)
//   posterior_coarse      stage 6 on Omega^R: r = beta^{1/2} nu + alpha^{1/2} xi with nu
//                         from eq. nuPerpendicular, then r' = r + sum_o (A^{1/2} - I) r on
//                         the 7x7 block of every observation (gathered, order fixed)
// All reductions use fixed trees, so results do not depend on scheduling.
#include <algorithm>

#include "internal.hpp"
#include "philox_dev.hpp"

namespace iewpf {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

constexpr int kWavesPerBlock = kThreads / 64;

// Wave reductions by a butterfly of lane exchanges: at every level both partners add (or
// compare) the same two values, so all lanes end with identical bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Fixed-order block sum of one double per thread (blockDim.x == kThreads): wave sums, then
// the kWavesPerBlock wave sums in wave order.  sh holds at least kWavesPerBlock doubles.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) r += sh[w];
  __syncthreads();  // sh is free again
  return r;
}

// Block minimum (exact in any order).
__device__ double block_min(double v, double* sh) {
  v = wave_min(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < kWavesPerBlock; ++w) r = fmin(r, sh[w]);
  __syncthreads();
  return r;
}

struct Mat2 {
  double a[4];
};

// particle i's innovations, S d and c_i (one workgroup)
__device__ __forceinline__ void innovation_body(
    int i, int n_obs, int max_obs, int nx, int ny, double H, const Mat2& S, double out_scale,
    const float* __restrict__ psi, const int32_t* __restrict__ cells, const double* __restrict__ y,
    double* __restrict__ sd, float* __restrict__ sdf, int ne4, double* __restrict__ cval,
    double* sh) {
  const size_t ncell = (size_t)nx * ny;
  const float* E = psi + (size_t)i * 3 * ncell;
  double phi = 0.0;
  for (int o = threadIdx.x; o < n_obs; o += kThreads) {
    const int j = cells[2 * o], k = cells[2 * o + 1];
    const size_t c = (size_t)k * nx + j;
    const double eta = E[c], hu = E[ncell + c], hv = E[2 * ncell + c];
    const double scale = (H + eta) / H;
    const double d0 = y[2 * o] * scale - hu;
    const double d1 = y[2 * o + 1] * scale - hv;
    const double s0 = S.a[0] * d0 + S.a[1] * d1;
    const double s1 = S.a[2] * d0 + S.a[3] * d1;
    sd[((size_t)i * max_obs + o) * 2] = s0;
    sd[((size_t)i * max_obs + o) * 2 + 1] = s1;
    if (sdf) {
      sdf[((size_t)o * ne4 + i) * 2] = static_cast<float>(s0);
      sdf[((size_t)o * ne4 + i) * 2 + 1] = static_cast<float>(s1);
    }
    phi += d0 * s0 + d1 * s1;
  }
  phi = block_sum(phi, sh);
  if (threadIdx.x == 0) cval[i] = out_scale * phi;
}

__global__ __launch_bounds__(kThreads) void innovation_kernel(
    int n_obs, int max_obs, int nx, int ny, double H, Mat2 S, double out_scale,
    const float* __restrict__ psi, const int32_t* __restrict__ cells, const double* __restrict__ y,
    double* __restrict__ sd, float* __restrict__ sdf, int ne4, double* __restrict__ cval) {
  __shared__ double sh[kThreads];
  innovation_body(blockIdx.x, n_obs, max_obs, nx, ny, H, S, out_scale, psi, cells, y, sd, sdf, ne4,
                  cval, sh);
}

// Normalised weights of the standard particle filter from log-weights (one workgroup):
// w_i = exp(l_i - max l) / sum_j exp(l_j - max l), the sum in a fixed order.
__global__ __launch_bounds__(kThreads) void sir_normalise_kernel(int ne, const double* __restrict__ logw,
                                                                 double* __restrict__ w) {
  __shared__ double sh[kWavesPerBlock];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < ne; i += kThreads) m = fmax(m, logw[i]);
  m = -block_min(-m, sh);
  double s = 0.0;
  for (int i = threadIdx.x; i < ne; i += kThreads) s += exp(logw[i] - m);
  s = block_sum(s, sh);
  for (int i = threadIdx.x; i < ne; i += kThreads) w[i] = exp(logw[i] - m) / s;
}

// Drifter observations (eq. drifterObservation): displacement over the observation interval
// times the equilibrium depth, plus noise from stream (step, tag 4, ens, particle word 1);
// the observed cell is the one holding the current position (eq. stateObservation).
__global__ void observe_drifters_kernel(int n, int nx, int ny, double dx, double dy, double H,
                                        double sigma, double dt_obs, uint64_t seed, uint64_t step,
                                        uint32_t ens, const double* __restrict__ pos_now,
                                        const double* __restrict__ pos_prev,
                                        int32_t* __restrict__ cells, double* __restrict__ y) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  const double px = pos_now[2 * d], py = pos_now[2 * d + 1];
  long long j = (long long)floor(px / dx) % nx;
  long long k = (long long)floor(py / dy) % ny;
  cells[2 * d] = (int32_t)(j < 0 ? j + nx : j);
  cells[2 * d + 1] = (int32_t)(k < 0 ? k + ny : k);
  double z[4];
  normals4((2 * d) / 4, step, 4u, ens, 1, seed, z);
  const int l = (2 * d) % 4;
  y[2 * d] = (px - pos_prev[2 * d]) / dt_obs * H + sigma * z[l];
  y[2 * d + 1] = (py - pos_prev[2 * d + 1]) / dt_obs * H + sigma * z[l + 1];
}

// grid (parts, ne): part q of particle i handles Philox blocks q*kThreads + t + k*stride
// (stride = parts*kThreads); partial sums go to part_dots[i][q][3] and are added in the
// fixed order q = 0.. by the sync kernel.  The host picks parts so that one pass covers
// the grid when it can (each thread then draws its normals once), at most kDotParts.
constexpr int kDotParts = 16;

// part q of particle i's draws and dot products (one workgroup)
__device__ __forceinline__ void rand_dots_body(int i, int q, int nr, int parts, uint64_t seed,
                                               uint64_t step, uint32_t ens, float* __restrict__ xi,
                                               float* __restrict__ nu,
                                               double* __restrict__ part_dots,
                                               const uint64_t* __restrict__ dyn, double* sh) {
  if (dyn) step += dyn[1];  // analysis index from device memory (captured graphs)
  float* X = xi + (size_t)i * nr;
  float* N = nu + (size_t)i * nr;
  double xx = 0.0, nn = 0.0, nxv = 0.0;
  const int nblk = (nr + 3) / 4;
  for (int b = q * kThreads + threadIdx.x; b < nblk; b += kThreads * parts) {
    double zx[4], zn[4];
    normals4(b, step, 2u, ens, i, seed, zx);
    normals4(b, step, 3u, ens, i, seed, zn);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int p = 4 * b + l;
      if (p < nr) {
        const float fx = static_cast<float>(zx[l]), fn = static_cast<float>(zn[l]);
        X[p] = fx;
        N[p] = fn;
        xx += (double)fx * fx;
        nn += (double)fn * fn;
        nxv += (double)fn * fx;
      }
    }
  }
  xx = block_sum(xx, sh);
  nn = block_sum(nn, sh);
  nxv = block_sum(nxv, sh);
  if (threadIdx.x == 0) {
    double* o = part_dots + ((size_t)i * parts + q) * 3;
    o[0] = xx;
    o[1] = nn;
    o[2] = nxv;
  }
}

__global__ __launch_bounds__(kThreads) void rand_dots_kernel(int nr, int parts, uint64_t seed,
                                                             uint64_t step, uint32_t ens,
                                                             float* __restrict__ xi,
                                                             float* __restrict__ nu,
                                                             double* __restrict__ part_dots,
                                                             const uint64_t* __restrict__ dyn) {
  __shared__ double sh[kThreads];
  rand_dots_body(blockIdx.y, blockIdx.x, nr, parts, seed, step, ens, xi, nu, part_dots, dyn, sh);
}

// Stages 1-3 in one launch: grid (parts + 1, ne); workgroup x = parts computes particle y's
// innovations, the others its draws (the two are independent).
__global__ __launch_bounds__(kThreads) void innov_draws_kernel(
    int n_obs, int max_obs, int nx, int ny, double H, Mat2 S, const float* __restrict__ psi,
    const int32_t* __restrict__ cells, const double* __restrict__ y, double* __restrict__ sd,
    float* __restrict__ sdf, int ne4, double* __restrict__ cval, int nr, int parts, uint64_t seed,
    uint64_t step, uint32_t ens, float* __restrict__ xi, float* __restrict__ nu, double* __restrict__ part_dots,
    const uint64_t* __restrict__ dyn) {
  __shared__ double sh[kThreads];
  if ((int)blockIdx.x == parts)
    innovation_body(blockIdx.y, n_obs, max_obs, nx, ny, H, S, 1.0, psi, cells, y, sd, sdf, ne4,
                    cval, sh);
  else
    rand_dots_body(blockIdx.y, blockIdx.x, nr, parts, seed, step, ens, xi, nu, part_dots, dyn, sh);
}


// (x - 1) - ln x for x = 1 + e, accurate for small e.
__device__ double xm1_minus_log(double e) {
  if (fabs(e) < 1e-2) {
    double s = 0.0, term = e * e;
    for (int k = 2; k < 24; ++k) {
      s += (k & 1) ? -term / k : term / k;
      term *= e;
    }
    return s;
  }
  return e - log1p(e);
}

// alpha solving (alpha - 1) gamma - N ln alpha = c* on the principal branch, i.e.
// alpha = -(N/gamma) W_0(-(gamma/N) e^{-gamma/N} e^{-c*/N}).  With y = -W_0 = alpha gamma/N:
// y - ln y = 1 + rho, rho = (gamma/N - 1 - ln(gamma/N)) + c*/N.  Halley iterations on
// delta = 1 - y near the branch point (rho < 1/2), on y otherwise.
// Stop once a Halley step is below 2^-44 of the iterate: convergence is cubic, so the
// iterate after such a step sits at the rounding floor of f (about 1e-13 relative near the
// branch point, where f cancels to O(d^2)); a tighter test can stall on rounding noise and
// run to the iteration cap.
constexpr double kHalleyStop = 0x1p-44;

__device__ double alpha_solve(double gamma, double cstar, double N) {
  const double x = gamma / N;
  const double cn = fmax(cstar, 0.0) / N;
  if (cn == 0.0 && x <= 1.0) return 1.0;
  const double rho = xm1_minus_log((gamma - N) / N) + cn;
  double y;
  if (rho <= 0.0) {
    y = 1.0;
  } else if (rho < 0.5) {
    const double p = sqrt(2.0 * rho);
    double d = p - p * p / 3.0 + 11.0 / 72.0 * p * p * p;  // branch-point series start
    for (int it = 0; it < 60; ++it) {
      const double om = 1.0 - d;
      const double f = -d - log1p(-d) - rho;
      const double f1 = d / om;
      const double f2 = 1.0 / (om * om);
      const double den = 2.0 * f1 * f1 - f * f2;
      const double step = den != 0.0 ? 2.0 * f * f1 / den : 0.0;
      double dn = d - step;
      if (dn <= 0.0) dn = 0.5 * d;
      if (dn >= 1.0) dn = 0.5 * (d + 1.0);
      const bool done = fabs(dn - d) <= kHalleyStop * d;
      d = dn;
      if (done) break;
    }
    y = 1.0 - d;
  } else {
    const double R = 1.0 + rho;
    y = exp(-R);
    for (int it = 0; it < 100; ++it) {
      const double g = y - log(y) - R;
      const double g1 = 1.0 - 1.0 / y;
      const double g2 = 1.0 / (y * y);
      const double den = 2.0 * g1 * g1 - g * g2;
      const double step = den != 0.0 ? 2.0 * g * g1 / den : 0.0;
      double yn = y - step;
      if (yn <= 0.0) yn = 0.5 * y;
      if (yn >= 1.0) yn = 0.5 * (y + 1.0);
      const bool done = fabs(yn - y) <= kHalleyStop * y;
      y = yn;
      if (done) break;
    }
  }
  return y / x;
}

// one_stage = 0: two-stage scheme (target = mean c, beta from eq. betaTwoStage, c* from eq.
// cistarTwoStage).  one_stage = 1: the original scheme of Appendix A (target = max c, eq.
// iewpf_targetWeight; no nu term, beta = 0; c* = target - c_i, eq. iewpfCStar); scal[0] then
// holds the target and scal[7] the particle that sets it.
__global__ __launch_bounds__(kThreads) void sync_kernel(int ne, double n_psi, double n_r,
                                                        int one_stage,
                                                        const double* __restrict__ cval,
                                                        const double* __restrict__ part_dots,
                                                        int parts, double* __restrict__ dots,
                                                        double* __restrict__ alpha,
                                                        double* __restrict__ cstar,
                                                        double* __restrict__ scal,
                                                        double* __restrict__ host_out) {
  __shared__ double sh[kWavesPerBlock];
  __shared__ double shb[kWavesPerBlock];
  __shared__ int shi[kWavesPerBlock];
  __shared__ double sh6[6][kWavesPerBlock];
  // the draws' dot products: the parts of each particle added in the fixed order q = 0..
  // (each thread sums and later reads only its own particles)
  for (int i = threadIdx.x; i < ne; i += kThreads) {
    // all parts loaded before the sums (parts <= kDotParts; the missing ones add +0)
    const double* o = part_dots + (size_t)i * parts * 3;
    double v[kDotParts][3];
#pragma unroll
    for (int q = 0; q < kDotParts; ++q)
#pragma unroll
      for (int r = 0; r < 3; ++r) v[q][r] = o[3 * min(q, parts - 1) + r];
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int q = 0; q < kDotParts; ++q) {
      const bool in = q < parts;
      a += in ? v[q][0] : 0.0;
      b += in ? v[q][1] : 0.0;
      c += in ? v[q][2] : 0.0;
    }
    dots[3 * i] = a;
    dots[3 * i + 1] = b;
    dots[3 * i + 2] = c;
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < ne; i += kThreads) s += cval[i];
  const double cmean = block_sum(s, sh) / ne;
  const double scale = n_psi / n_r;
  // two-stage: beta = min_i ((cbar - c_i)/zeta_i + 1); one-stage: the largest c_i (as the
  // minimum of -c_i); argmin with the smallest index on ties
  double bmin = 1e300;
  int imin = 0x7fffffff;
  for (int i = threadIdx.x; i < ne; i += kThreads) {
    const double zeta = dots[3 * i + 1] * scale;
    const double b = one_stage ? -cval[i] : (cmean - cval[i]) / zeta + 1.0;
    if (b < bmin || (b == bmin && i < imin)) {
      bmin = b;
      imin = i;
    }
  }
  // smallest (b, i) in lexicographic order: exact, the same in every lane
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double b2 = __shfl_xor(bmin, o, 64);
    const int i2 = __shfl_xor(imin, o, 64);
    if (b2 < bmin || (b2 == bmin && i2 < imin)) {
      bmin = b2;
      imin = i2;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    shb[threadIdx.x >> 6] = bmin;
    shi[threadIdx.x >> 6] = imin;
  }
  __syncthreads();
  double bb = shb[0];
  int ii = shi[0];
  for (int w = 1; w < kWavesPerBlock; ++w) {
    if (shb[w] < bb || (shb[w] == bb && shi[w] < ii)) {
      bb = shb[w];
      ii = shi[w];
    }
  }
  const double beta = one_stage ? 0.0 : bb;
  const double cbar = one_stage ? -bb : cmean;  // the target weight
  const int argmin = ii;
  double amin = 1e300, amax = -1e300, csmax = 0.0, cmin = 1e300, cmax = -1e300;
  double first_bad = 1e300;  // smallest particle with a non-finite scalar
  for (int i = threadIdx.x; i < ne; i += kThreads) {
    const double gamma = dots[3 * i] * scale;
    const double zeta = dots[3 * i + 1] * scale;
    const double cs = fmax(0.0, one_stage ? cbar - cval[i] : cbar - cval[i] - (beta - 1.0) * zeta);
    const double a = (one_stage || beta > 0.0) ? alpha_solve(gamma, cs, n_psi) : 0.0;
    cstar[i] = cs;
    alpha[i] = a;
    amin = fmin(amin, a);
    amax = fmax(amax, a);
    csmax = fmax(csmax, cs);
    cmin = fmin(cmin, cval[i]);
    cmax = fmax(cmax, cval[i]);
    // fmax/fmin drop NaN operands, so non-finite values are caught here, not by the ranges
    const bool finite = isfinite(cval[i]) && isfinite(gamma) && isfinite(zeta) && isfinite(cs) &&
                        isfinite(a);
    if (!finite) first_bad = fmin(first_bad, (double)i);
  }
  // min / max reductions (order independent), all six in one exchange through LDS
  double outv[6] = {amin, -amax, -csmax, cmin, -cmax, first_bad};
#pragma unroll
  for (int q = 0; q < 6; ++q) outv[q] = wave_min(outv[q]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 6; ++q) sh6[q][threadIdx.x >> 6] = outv[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double r = sh6[q][0];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) r = fmin(r, sh6[q][w]);
    outv[q] = r;
  }
  if (threadIdx.x == 0) {
    // status words read by the posterior and update kernels (which write nothing when an
    // error bit is set) and by the host after the analysis
    int32_t* st = reinterpret_cast<int32_t*>(scal + kScalStatus);
    int flags = 0;
    if (outv[5] < 1e300) flags |= kStatNonfiniteScalar;
    if (!one_stage && !(beta > 0.0)) flags |= kStatBeta;
    st[0] = flags;
    st[1] = outv[5] < 1e300 ? static_cast<int32_t>(outv[5]) : -1;
    st[2] = 0;           // set by the update kernel when a written value is not finite
    st[3] = 0x7fffffff;  // smallest such particle (atomic minimum)
    scal[0] = cbar;
    scal[1] = beta;
    scal[2] = outv[0];
    scal[3] = -outv[1];
    scal[4] = -outv[2];
    scal[5] = outv[3];
    scal[6] = -outv[4];
    scal[7] = static_cast<double>(argmin);
    if (host_out) {
      // the scalars and status words for the host (pinned, mapped): no copy after the
      // analysis; the fifth int32 after the scalars is the update's "read the device
      // status" flag
      for (int q = 0; q < kScalStatus; ++q) host_out[q] = scal[q];
      int32_t* hs = reinterpret_cast<int32_t*>(host_out + kScalStatus);
      hs[0] = flags;
      hs[1] = st[1];
      hs[2] = 0;
      hs[3] = 0x7fffffff;
      hs[4] = 0;
    }
  }
}

// Full innovation covariance (all observations together instead of independent 2x2 blocks).
// Entry ((o2, a), (o, b)) of the chain's H Q H^T is component a (hu, hv) of the pull window
// of unit vector e_b, read at the offset of observation o2's cell from observation o's cell
// (zero beyond the window's reach); the matrix is symmetrised and R = sigma^2 I added.
__global__ void hqht_full_kernel(int n_obs, int nx, int ny, int rx, int ry, int wx, int wy,
                                 const double* __restrict__ win, const int32_t* __restrict__ cells,
                                 double sigma2, double* __restrict__ M) {
  const int n = 2 * n_obs;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int r = t / n, col = t - r * n;
  const size_t plane = (size_t)wx * wy;
  auto entry = [&](int rr, int cc) -> double {
    const int o2 = rr >> 1, a = rr & 1, o = cc >> 1, b = cc & 1;
    int dj = cells[2 * o2] - cells[2 * o], dk = cells[2 * o2 + 1] - cells[2 * o + 1];
    int ix, iy;
    if (rx >= 0) {
      dj = dj > nx / 2 ? dj - nx : (dj < -(nx / 2) ? dj + nx : dj);
      if (dj < -rx || dj > rx) return 0.0;
      ix = dj + rx;
    } else {
      ix = wrapi(dj, nx);
    }
    if (ry >= 0) {
      dk = dk > ny / 2 ? dk - ny : (dk < -(ny / 2) ? dk + ny : dk);
      if (dk < -ry || dk > ry) return 0.0;
      iy = dk + ry;
    } else {
      iy = wrapi(dk, ny);
    }
    return win[(size_t)(b * 3 + 1 + a) * plane + (size_t)iy * wx + ix];
  };
  M[t] = 0.5 * (entry(r, col) + entry(col, r)) + (r == col ? sigma2 : 0.0);
}

// Cholesky factor of a symmetric positive definite A [n][n] (n <= kCholThreads) in place,
// one workgroup, float64.  Right-looking in panels of kCholPanel columns: the panel (rows
// p0 .. n-1) is factored in LDS, written back, and the trailing lower triangle is updated
// once per panel with kCholPanel-term dot products read from LDS.  On return the lower
// triangle holds L and the strict upper triangle L^T (row r of the upper triangle is column
// r of L), so both triangular solves read rows.  status[0] = 1 when a pivot is not positive.
constexpr int kCholThreads = 1024;
constexpr int kCholPanel = 16;
constexpr int kCholStride = kCholPanel + 1;  // LDS row stride (doubles)
__global__ __launch_bounds__(kCholThreads) void chol_factor_kernel(int n, double* __restrict__ A,
                                                                   int32_t* __restrict__ status) {
  extern __shared__ double P[];  // [n - p0][kCholStride]
  const int tid = threadIdx.x;
  const int sub = tid & (kCholPanel - 1), grp = tid / kCholPanel;  // 64 row groups of 16 lanes
  constexpr int kGroups = kCholThreads / kCholPanel;
  bool bad = false;
  for (int p0 = 0; p0 < n; p0 += kCholPanel) {
    const int pw = min(kCholPanel, n - p0);
    const int m = n - p0;
    for (int i = grp; i < m; i += kGroups)
      if (sub < pw) P[i * kCholStride + sub] = A[(size_t)(p0 + i) * n + p0 + sub];
    __syncthreads();
    for (int c = 0; c < pw; ++c) {
      const double d = P[c * kCholStride + c];
      if (!(d > 0.0)) bad = true;
      const double piv = sqrt(d > 0.0 ? d : 1.0);
      __syncthreads();  // every thread has read the pivot before it is replaced
      for (int i = c + tid; i < m; i += kCholThreads)
        P[i * kCholStride + c] = i == c ? piv : P[i * kCholStride + c] / piv;
      __syncthreads();
      const int k = c + 1 + sub;  // remaining panel columns, rows i >= k
      if (k < pw) {
        const double lk = P[k * kCholStride + c];
        for (int i = k + grp; i < m; i += kGroups)
          P[i * kCholStride + k] -= P[i * kCholStride + c] * lk;
      }
      __syncthreads();
    }
    // write back L (lower) and L^T (upper rows p0 .. p0+pw-1)
    for (int i = grp; i < m; i += kGroups) {
      if (sub < pw && i >= sub) {
        const double v = P[i * kCholStride + sub];
        A[(size_t)(p0 + i) * n + p0 + sub] = v;
        A[(size_t)(p0 + sub) * n + p0 + i] = v;
      }
    }
    // trailing update of the lower triangle right of the panel
    const int q0 = p0 + pw;
    const int tx = tid & 31, ty = tid >> 5;
    for (int i = q0 + ty; i < n; i += 32) {
      const double* Pi = P + (i - p0) * kCholStride;
      double* row = A + (size_t)i * n;
      for (int k = q0 + tx; k <= i; k += 32) {
        const double* Pk = P + (k - p0) * kCholStride;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kCholPanel; ++c)
          if (c < pw) acc += Pi[c] * Pk[c];
        row[k] -= acc;
      }
    }
    __syncthreads();
  }
  if (tid == 0) status[0] = 0;
  __syncthreads();
  if (bad && tid == 0) status[0] = 1;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Solves A x = b with the factor above for every right-hand side, one wave each:
// L y = b by forward substitution, then L^T x = y by back substitution, both column by
// column (x_j fixed, then subtracted from every later row), so every step reads one row of
// a triangle; lane l keeps rows l, l + 64, ... (S slots).  The row of the next step is
// loaded during the current one.  out = x (= S b), cval = y^T y (= b^T S b).
// rhs == nullptr: b = e_w for wave w (the columns of S = A^{-1}).
template <int S>
__global__ __launch_bounds__(256) void chol_solve_kernel(int n, int nrhs, const double* __restrict__ A,
                                                         const double* __restrict__ rhs, int rhs_stride,
                                                         double* __restrict__ out, int out_stride,
                                                         double* __restrict__ cval) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (w >= nrhs) return;
  double b[S];
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int r = t * 64 + lane;
    b[t] = 0.0;
    if (r < n) b[t] = rhs ? rhs[(size_t)w * rhs_stride + r] : (r == w ? 1.0 : 0.0);
  }
  double ss = 0.0;
  double cur[S], nxt[S];
  // forward: y_j = b_j / L_jj; b_r -= L_rj y_j (r > j), L_rj = A[j][r] (upper row j)
#pragma unroll
  for (int t = 0; t < S; ++t) {
    cur[t] = t * 64 + lane < n ? A[t * 64 + lane] : 0.0;
    nxt[t] = 0.0;
  }
#pragma unroll
  for (int js = 0; js < S; ++js) {
    if (js * 64 < n) {
      for (int jl = 0; jl < 64; ++jl) {
        const int j = js * 64 + jl;
        if (j >= n) break;
        if (j + 1 < n) {
#pragma unroll
          for (int t = js; t < S; ++t) {
            const int r = t * 64 + lane;
            nxt[t] = r < n ? A[(size_t)(j + 1) * n + r] : 0.0;
          }
        }
        const double yj = readlane_f64(b[js], jl) / readlane_f64(cur[js], jl);
        ss += yj * yj;
        if (lane == jl) b[js] = yj;
#pragma unroll
        for (int t = js; t < S; ++t) {
          const int r = t * 64 + lane;
          if (r > j && r < n) b[t] -= cur[t] * yj;
        }
#pragma unroll
        for (int t = js; t < S; ++t) cur[t] = nxt[t];
      }
    }
  }
  // backward: x_j = y_j / L_jj; y_r -= L_jr x_j (r < j), L_jr = A[j][r] (lower row j)
#pragma unroll
  for (int t = 0; t < S; ++t)
    cur[t] = t * 64 + lane < n ? A[(size_t)(n - 1) * n + t * 64 + lane] : 0.0;
#pragma unroll
  for (int js = S - 1; js >= 0; --js) {
    if (js * 64 < n) {
      for (int jl = 63; jl >= 0; --jl) {
        const int j = js * 64 + jl;
        if (j >= n) continue;
        if (j > 0) {
#pragma unroll
          for (int t = 0; t <= js; ++t) {
            const int r = t * 64 + lane;
            nxt[t] = r < n ? A[(size_t)(j - 1) * n + r] : 0.0;
          }
        }
        const double xj = readlane_f64(b[js], jl) / readlane_f64(cur[js], jl);
        if (lane == jl) b[js] = xj;
#pragma unroll
        for (int t = 0; t <= js; ++t) {
          const int r = t * 64 + lane;
          if (r < j) b[t] -= cur[t] * xj;
        }
#pragma unroll
        for (int t = 0; t <= js; ++t) cur[t] = nxt[t];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int r = t * 64 + lane;
    if (r < n) out[(size_t)w * out_stride + r] = b[t];
  }
  if (cval && lane == 0) cval[w] = ss;
}

// SD[p][r] = sum_c S[r][c] D[p][c] for every particle p and row r of the full S [n][n]
// (rows of D and SD are `stride` apart): 16 x 16 tiles of (row, particle), c in chunks of 32
// staged in LDS, each sum in increasing c.  SDf receives the same values in float32,
// observation-major ([r / 2][ne4][2]).
__global__ __launch_bounds__(256) void sd_gemm_kernel(int n, int ne, int stride, int ne4,
                                                      const double* __restrict__ S,
                                                      const double* __restrict__ D,
                                                      double* __restrict__ SD,
                                                      float* __restrict__ SDf) {
  __shared__ double Ts[16][33], Td[16][33];
  const int tr = threadIdx.x & 15, tp = threadIdx.x >> 4;
  const int r0 = blockIdx.x * 16, p0 = blockIdx.y * 16;
  double acc = 0.0;
  for (int c0 = 0; c0 < n; c0 += 32) {
    for (int e = threadIdx.x; e < 512; e += 256) {
      const int a = e >> 5, cc = e & 31, c = c0 + cc;
      Ts[a][cc] = (r0 + a < n && c < n) ? S[(size_t)(r0 + a) * n + c] : 0.0;
      Td[a][cc] = (p0 + a < ne && c < n) ? D[(size_t)(p0 + a) * stride + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < 32; ++cc) acc += Ts[tr][cc] * Td[tp][cc];
    __syncthreads();
  }
  if (r0 + tr < n && p0 + tp < ne) {
    const int r = r0 + tr, p = p0 + tp;
    SD[(size_t)p * stride + r] = acc;
    SDf[((size_t)(r >> 1) * ne4 + p) * 2 + (r & 1)] = static_cast<float>(acc);
  }
}

// c_p = d_p^T (S d_p), one workgroup per particle, fixed-order sum.
__global__ __launch_bounds__(kThreads) void dot_rows_kernel(int n, int stride,
                                                            const double* __restrict__ D,
                                                            const double* __restrict__ SD,
                                                            double* __restrict__ cval) {
  __shared__ double sh[kThreads];
  const size_t o = (size_t)blockIdx.x * stride;
  double v = 0.0;
  for (int r = threadIdx.x; r < n; r += kThreads) v += D[o + r] * SD[o + r];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) cval[blockIdx.x] = v;
}

// Posterior random field on the coarse grid, r_i + (A^{1/2} - I) r_i on each observation's
// 7x7 block, in two passes: one wave per (observation, particle) forms the block product
// v = (A^{1/2} - I) r_block (each row summed in increasing block index), then one work-item
// per (coarse point, particle) adds the rows of the blocks that contain the point to r
// (ascending observations).
struct PostCoef {
  double a, sb, sa;
};
__device__ __forceinline__ PostCoef post_coef(int i, const double* __restrict__ dots,
                                              const double* __restrict__ alpha,
                                              const double* __restrict__ scal) {
  const double xx = dots[3 * i], nn = dots[3 * i + 1], nxv = dots[3 * i + 2];
  PostCoef k;
  k.a = nxv / xx;
  const double sperp = sqrt(nn / (nn - k.a * nxv));
  const double beta = scal[1];
  k.sb = sqrt(fmax(beta, 0.0)) * sperp;
  k.sa = sqrt(alpha[i]);
  return k;
}
__device__ __forceinline__ double post_r(const PostCoef& k, float x, float n) {
  const double xv = x, nv = n;
  return k.sb * (nv - k.a * xv) + k.sa * xv;
}

// One wave per (observation, kPostGroup particles): lanes < kPostGroup form the particles'
// coefficients (the group's first observation stores them for the point pass), lanes m < 49
// then load r at block point m for every particle of the group, and lane m forms row m of
// (A^{1/2} - I) r for all of them (independent sum chains, each in increasing block index).
constexpr int kPostGroup = 16;
__global__ __launch_bounds__(kWave) void posterior_blocks_kernel(
    CoarseConst C, int ne, int n_obs, int max_obs, const int32_t* __restrict__ cells,
    const float* __restrict__ xi, const float* __restrict__ nu, const double* __restrict__ dots,
    const double* __restrict__ alpha, const double* __restrict__ scal,
    const float* __restrict__ dmat, double* __restrict__ vblk, double* __restrict__ coef) {
  __shared__ double rb[kPostGroup][kBlockN];
  __shared__ double kc[kPostGroup][3];
  if (reinterpret_cast<const int32_t*>(scal + kScalStatus)[0] & kStatSkipUpdate) return;
  const int o = blockIdx.x;
  const int i0 = blockIdx.y * kPostGroup;
  const int ng = min(kPostGroup, ne - i0);
  const int nr = C.nrx * C.nry;
  const int m = threadIdx.x;
  if (m < kPostGroup) {  // a short group repeats its last particle
    const PostCoef k = post_coef(i0 + min(m, ng - 1), dots, alpha, scal);
    kc[m][0] = k.a;
    kc[m][1] = k.sb;
    kc[m][2] = k.sa;
    if (o == 0 && m < ng) {
      coef[3 * (i0 + m)] = k.a;
      coef[3 * (i0 + m) + 1] = k.sb;
      coef[3 * (i0 + m) + 2] = k.sa;
    }
  }
  __syncthreads();
  const bool active = m < kBlockN && n_obs > 0;
  if (active) {
    // block point m: offset (m / 7 - 3, m % 7 - 3) from the observation's coarse cell
    const int ao = cells[2 * o] / C.c, bo = cells[2 * o + 1] / C.c;
    const int q = wrapi(bo + m / 7 - 3, C.nry) * C.nrx + wrapi(ao + m % 7 - 3, C.nrx);
    float xv[kPostGroup], nv[kPostGroup];
#pragma unroll
    for (int g = 0; g < kPostGroup; ++g) {
      const int i = i0 + min(g, ng - 1);
      xv[g] = xi[(size_t)i * nr + q];
      nv[g] = nu[(size_t)i * nr + q];
    }
#pragma unroll
    for (int g = 0; g < kPostGroup; ++g) {
      PostCoef k;
      k.a = kc[g][0];
      k.sb = kc[g][1];
      k.sa = kc[g][2];
      rb[g][m] = post_r(k, xv[g], nv[g]);
    }
  }
  __syncthreads();
  if (!active) return;
  float d[kBlockN];
#pragma unroll
  for (int b = 0; b < kBlockN; ++b) d[b] = dmat[m * kBlockN + b];
  double v[kPostGroup];
#pragma unroll
  for (int g = 0; g < kPostGroup; ++g) v[g] = 0.0;
#pragma unroll
  for (int b = 0; b < kBlockN; ++b) {
    const double db = d[b];
#pragma unroll
    for (int g = 0; g < kPostGroup; ++g) v[g] += db * rb[g][b];
  }
  for (int g = 0; g < ng; ++g) vblk[((size_t)(i0 + g) * max_obs + o) * kBlockN + m] = v[g];
}

// One work-item per coarse point for kPtGroup particles: the point's block entries are read
// once for the group.
constexpr int kPtGroup = 8;
__global__ __launch_bounds__(256) void posterior_points_kernel(
    CoarseConst C, int ne, int max_obs, const float* __restrict__ xi,
    const float* __restrict__ nu, const double* __restrict__ coef,
    const double* __restrict__ scal, const int32_t* __restrict__ pt_off,
    const int32_t* __restrict__ pt_ent, const double* __restrict__ vblk,
    float* __restrict__ rout) {
  if (reinterpret_cast<const int32_t*>(scal + kScalStatus)[0] & kStatSkipUpdate) return;
  const int nr = C.nrx * C.nry;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * kPtGroup;
  if (p >= nr) return;
  const int ng = min(kPtGroup, ne - i0);
  double acc[kPtGroup];
#pragma unroll
  for (int g = 0; g < kPtGroup; ++g) {
    const int i = i0 + min(g, ng - 1);
    PostCoef k;
    k.a = coef[3 * i];
    k.sb = coef[3 * i + 1];
    k.sa = coef[3 * i + 2];
    acc[g] = post_r(k, xi[(size_t)i * nr + p], nu[(size_t)i * nr + p]);
  }
  const int t1 = pt_off[p + 1];
  for (int t = pt_off[p]; t < t1; ++t) {
    const int e = pt_ent[t];  // (observation << 8) | this point's position in the block
    const size_t off = (size_t)(e >> 8) * kBlockN + (e & 255);
#pragma unroll
    for (int g = 0; g < kPtGroup; ++g)
      acc[g] += vblk[(size_t)(i0 + min(g, ng - 1)) * max_obs * kBlockN + off];
  }
  for (int g = 0; g < ng; ++g) rout[(size_t)(i0 + g) * nr + p] = static_cast<float>(acc[g]);
}

__global__ void observe_kernel(int n_obs, int nx, int ny, double H, double sigma, uint64_t seed,
                               uint64_t step, uint32_t ens, const float* __restrict__ truth,
                               const int32_t* __restrict__ cells, double* __restrict__ y) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_obs) return;
  const size_t ncell = (size_t)nx * ny;
  const int j = cells[2 * o], k = cells[2 * o + 1];
  const size_t c = (size_t)k * nx + j;
  const double eta = truth[c], hu = truth[ncell + c], hv = truth[2 * ncell + c];
  const double s = H / (H + eta);
  double z[4];
  normals4((2 * o) / 4, step, 4u, ens, 0, seed, z);
  const int l = (2 * o) % 4;
  y[2 * o] = hu * s + sigma * z[l];
  y[2 * o + 1] = hv * s + sigma * z[l + 1];
}

__global__ __launch_bounds__(256) void cfl_kernel(size_t n_cells_total, size_t ncell, float H, float g,
                                                  const float* __restrict__ psi,
                                                  unsigned* __restrict__ out) {
  float sx = 0.0f, sy = 0.0f;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n_cells_total;
       t += (size_t)gridDim.x * blockDim.x) {
    const size_t i = t / ncell, c = t - i * ncell;
    const float* E = psi + i * 3 * ncell;
    const float h = H + E[c];
    const float cw = sqrtf(g * h);
    sx = fmaxf(sx, fabsf(E[ncell + c] / h) + cw);
    sy = fmaxf(sy, fabsf(E[2 * ncell + c] / h) + cw);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sx = fmaxf(sx, __shfl_down(sx, off, 64));
    sy = fmaxf(sy, __shfl_down(sy, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, __float_as_uint(sx));
    atomicMax(out + 1, __float_as_uint(sy));
  }
}

// Bilinear velocity of one particle's state at position (px, py) (metres, unwrapped).
// Velocity of the state Ea + w (Eb - Ea) (Eb = Ea, w = 0: the state Ea itself).
__device__ void velocity_at(const float* __restrict__ Ea, const float* __restrict__ Eb, double w,
                            int nx, int ny, double dx, double dy, double H, double px, double py,
                            double& u, double& v) {
  const size_t ncell = (size_t)nx * ny;
  const double fx = px / dx - 0.5, fy = py / dy - 0.5;
  const double fj = floor(fx), fk = floor(fy);
  const double tx = fx - fj, ty = fy - fk;
  long long j0 = (long long)fj, k0 = (long long)fk;
  j0 %= nx;
  if (j0 < 0) j0 += nx;
  k0 %= ny;
  if (k0 < 0) k0 += ny;
  const int j1 = (int)((j0 + 1) % nx), k1 = (int)((k0 + 1) % ny);
  const int js[2] = {(int)j0, j1}, ks[2] = {(int)k0, k1};
  const double wxs[2] = {1.0 - tx, tx}, wys[2] = {1.0 - ty, ty};
  u = 0.0;
  v = 0.0;
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) {
      const size_t c = (size_t)ks[b] * nx + js[a];
      double f[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double ea = Ea[q * ncell + c];
        f[q] = ea + w * ((double)Eb[q * ncell + c] - ea);
      }
      const double h = H + f[0];
      const double wt = wxs[a] * wys[b];
      u += wt * (f[1] / h);
      v += wt * (f[2] / h);
    }
}

__global__ void drift_k1_kernel(int ne, int nd, int nx, int ny, double dx, double dy, double H,
                                double dt, const float* __restrict__ psi,
                                const float* __restrict__ psi_b, double w,
                                const double* __restrict__ pos, double* __restrict__ k1,
                                double* __restrict__ pstar) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne * nd) return;
  const int i = t / nd;
  const float* E = psi + (size_t)i * 3 * nx * ny;
  const float* Eb = psi_b + (size_t)i * 3 * nx * ny;
  double u, v;
  velocity_at(E, Eb, w, nx, ny, dx, dy, H, pos[2 * t], pos[2 * t + 1], u, v);
  k1[2 * t] = u;
  k1[2 * t + 1] = v;
  pstar[2 * t] = pos[2 * t] + dt * u;
  pstar[2 * t + 1] = pos[2 * t + 1] + dt * v;
}

__global__ void drift_k2_kernel(int ne, int nd, int nx, int ny, double dx, double dy, double H,
                                double dt, const float* __restrict__ psi,
                                const float* __restrict__ psi_b, double w, double* __restrict__ pos,
                                const double* __restrict__ k1, const double* __restrict__ pstar,
                                double* __restrict__ traj) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne * nd) return;
  const int i = t / nd;
  const float* E = psi + (size_t)i * 3 * nx * ny;
  const float* Eb = psi_b + (size_t)i * 3 * nx * ny;
  double u, v;
  velocity_at(E, Eb, w, nx, ny, dx, dy, H, pstar[2 * t], pstar[2 * t + 1], u, v);
  const double px = pos[2 * t] + 0.5 * dt * (k1[2 * t] + u);
  const double py = pos[2 * t + 1] + 0.5 * dt * (k1[2 * t + 1] + v);
  pos[2 * t] = px;
  pos[2 * t + 1] = py;
  if (traj) {
    traj[2 * t] = px;
    traj[2 * t + 1] = py;
  }
}

// Residual resampling (Section "Standard particle filter"), one work-item: the decisions
// are integer and sequential over at most a few thousand particles.
// scal != nullptr (the SIR analysis): also writes the analysis scalars (c_min / c_max =
// range of -2 l_i, argmin_beta = the particle of largest weight, the IEWPF fields 0) and the
// status words; a non-finite log-weight flags the analysis and keeps the ensemble as it is.
__global__ void resample_kernel(int ne, uint64_t seed, uint64_t step, uint32_t ens,
                                const double* __restrict__ logw, int32_t* __restrict__ parents,
                                int32_t* __restrict__ counts, double* __restrict__ cum,
                                double* __restrict__ scal) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (scal) {
    int bad = -1, best = 0;
    double lo = logw[0], hi = logw[0];
    for (int i = 0; i < ne; ++i) {
      if (!isfinite(logw[i]) && bad < 0) bad = i;
      if (logw[i] > logw[best]) best = i;
      lo = fmin(lo, logw[i]);
      hi = fmax(hi, logw[i]);
    }
    for (int q = 0; q < 5; ++q) scal[q] = 0.0;
    scal[5] = -2.0 * hi;
    scal[6] = -2.0 * lo;
    scal[7] = (double)best;
    int32_t* st = reinterpret_cast<int32_t*>(scal + kScalStatus);
    st[0] = bad >= 0 ? kStatNonfiniteScalar : 0;
    st[1] = bad;
    st[2] = 0;
    st[3] = 0x7fffffff;
    if (bad >= 0) {
      for (int i = 0; i < ne; ++i) parents[i] = i;
      return;
    }
  }
  double m = logw[0];
  for (int i = 1; i < ne; ++i) m = fmax(m, logw[i]);
  double s = 0.0;
  for (int i = 0; i < ne; ++i) s += exp(logw[i] - m);
  if (!(s > 0.0) || !isfinite(s)) {  // no usable weights: keep the ensemble as it is
    for (int i = 0; i < ne; ++i) parents[i] = i;
    return;
  }
  // copies floor(N w_i); cum[i] = residuals r_0 + ... + r_i, summed left to right
  int used = 0;
  double total = 0.0, acc = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double x = (double)ne * exp(logw[i] - m) / s;
    const double n = (x >= 0.0 && x <= (double)ne) ? floor(x) : 0.0;
    counts[i] = (int)n;
    used += (int)n;
    total += (x >= 0.0 && x <= (double)ne) ? x - n : 0.0;
    acc += x - floor(x);
    cum[i] = acc;
  }
  // residual draws by inverse CDF: the first i with target < cum[i] (cum is non-decreasing)
  const int n_res = used <= ne ? ne - used : 0;
  for (int kdraw = 0; kdraw < n_res; ++kdraw) {
    const U64x4 w = philox4x64_10((uint64_t)(kdraw / 4), step, stream_word(6u, ens), 0, seed, 0);
    const uint64_t words[4] = {w.x0, w.x1, w.x2, w.x3};
    const double u = (double)(words[kdraw % 4] >> 11) * 0x1.0p-53;
    const double target = u * total;
    int lo = 0, hi = ne;  // search [lo, hi)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (target < cum[mid])
        hi = mid;
      else
        lo = mid + 1;
    }
    counts[lo < ne ? lo : ne - 1] += 1;
  }
  int t = 0;
  for (int i = 0; i < ne; ++i)
    for (int c = 0; c < counts[i] && t < ne; ++c) parents[t++] = i;
  for (; t < ne; ++t) parents[t] = ne - 1;  // unreachable when the counts sum to ne
}

// one workgroup per ensemble; workgroup 0 also copies the counters
__global__ __launch_bounds__(256) void batch_stage_in_kernel(BatchStageIn a) {
  const int e = blockIdx.x;
  const double* __restrict__ src = a.y_src[e];
  double* __restrict__ dst = a.y_dst[e];
  for (int i = threadIdx.x; i < a.n_y[e]; i += blockDim.x) dst[i] = src[i];
  if (e == 0 && a.dyn_src && threadIdx.x < 2) a.dyn_dst[threadIdx.x] = a.dyn_src[threadIdx.x];
}

__global__ __launch_bounds__(64) void batch_status_kernel(BatchStatusOut a, int n) {
  const int t = threadIdx.x;
  if (t < 4 * n) a.dst[t] = a.src[t >> 2][t & 3];
}

__global__ void gather_kernel(size_t per_particle4, const int32_t* __restrict__ parents,
                              const float4* __restrict__ in, float4* __restrict__ out) {
  const int i = blockIdx.y;
  const float4* src = in + (size_t)parents[i] * per_particle4;
  float4* dst = out + (size_t)i * per_particle4;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < per_particle4;
       t += (size_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

}  // namespace

void launch_innovation(int ne, int n_obs, int max_obs, int nx, int ny, double H, const double S[4],
                       const float* psi, const int32_t* cells, const double* y, double* sd,
                       float* sdf, double* cval, hipStream_t s, double out_scale) {
  Mat2 M{{S[0], S[1], S[2], S[3]}};
  hipLaunchKernelGGL(innovation_kernel, dim3(ne), dim3(kThreads), 0, s, n_obs, max_obs, nx, ny, H,
                     M, out_scale, psi, cells, y, sd, sdf, sd_float_stride(ne), cval);
}

void launch_sir_normalise(int ne, const double* logw, double* w, hipStream_t s) {
  hipLaunchKernelGGL(sir_normalise_kernel, dim3(1), dim3(kThreads), 0, s, ne, logw, w);
}

void launch_observe_drifters(int n, int nx, int ny, double dx, double dy, double H, double sigma,
                             double dt_obs, uint64_t seed, uint64_t step, uint32_t ens,
                             const double* pos_now, const double* pos_prev, int32_t* cells,
                             double* y, hipStream_t s) {
  hipLaunchKernelGGL(observe_drifters_kernel, dim3((n + 127) / 128), dim3(128), 0, s, n, nx, ny, dx,
                     dy, H, sigma, dt_obs, seed, step, ens, pos_now, pos_prev, cells, y);
}

int rand_dots_parts() { return kDotParts; }

int rand_dots_parts_for(int nr) {
  const int nblk = (nr + 3) / 4;
  return std::min(kDotParts, std::max(1, (nblk + kThreads - 1) / kThreads));
}

void launch_rand_dots(int ne, int nr, uint64_t seed, uint64_t step, uint32_t ens, float* xi,
                      float* nu, double* part_dots, hipStream_t s, const uint64_t* dyn) {
  const int parts = rand_dots_parts_for(nr);
  hipLaunchKernelGGL(rand_dots_kernel, dim3(parts, ne), dim3(kThreads), 0, s, nr, parts, seed, step,
                     ens, xi, nu, part_dots, dyn);
}

void launch_innov_draws(int ne, int n_obs, int max_obs, int nx, int ny, double H,
                        const double S[4], const float* psi, const int32_t* cells, const double* y,
                        double* sd, float* sdf, double* cval, int nr, uint64_t seed, uint64_t step,
                        uint32_t ens, float* xi, float* nu, double* part_dots, hipStream_t s,
                        const uint64_t* dyn) {
  Mat2 M{{S[0], S[1], S[2], S[3]}};
  const int parts = rand_dots_parts_for(nr);
  hipLaunchKernelGGL(innov_draws_kernel, dim3(parts + 1, ne), dim3(kThreads), 0, s, n_obs, max_obs,
                     nx, ny, H, M, psi, cells, y, sd, sdf, sd_float_stride(ne), cval, nr, parts,
                     seed, step, ens, xi, nu, part_dots, dyn);
}

void launch_sync(int ne, int nr, double n_psi, int one_stage, const double* cval,
                 const double* part_dots, double* dots, double* alpha, double* cstar,
                 double* scal, double* host_out, hipStream_t s) {
  hipLaunchKernelGGL(sync_kernel, dim3(1), dim3(kThreads), 0, s, ne, n_psi, (double)nr, one_stage,
                     cval, part_dots, rand_dots_parts_for(nr), dots, alpha, cstar, scal, host_out);
}

void launch_posterior_coarse(const CoarseConst& C, int ne, int n_obs, int max_obs,
                             const int32_t* cells, const float* xi, const float* nu,
                             const double* dots, const double* alpha, const double* scal,
                             const float* dmat, const int32_t* pt_off, const int32_t* pt_ent,
                             double* vblk, double* coef, float* rout, hipStream_t s) {
  // the point pass reads the coefficients the block pass stores with its first observation:
  // without observations one block pass column runs that only stores them
  const dim3 grid(std::max(1, n_obs), (ne + kPostGroup - 1) / kPostGroup);
  hipLaunchKernelGGL(posterior_blocks_kernel, grid, dim3(kWave), 0, s, C, ne, n_obs, max_obs,
                     cells, xi, nu, dots, alpha, scal, dmat, vblk, coef);
  const int nr = C.nrx * C.nry;
  hipLaunchKernelGGL(posterior_points_kernel, dim3((nr + 255) / 256, (ne + kPtGroup - 1) / kPtGroup),
                     dim3(256), 0, s, C, ne, max_obs, xi, nu, coef, scal, pt_off, pt_ent, vblk,
                     rout);
}

void launch_hqht_full(int n_obs, int nx, int ny, int rx, int ry, int wx, int wy, const double* win,
                      const int32_t* cells, double sigma2, double* M, hipStream_t s) {
  const int n = 2 * n_obs;
  hipLaunchKernelGGL(hqht_full_kernel, dim3((n * n + 255) / 256), dim3(256), 0, s, n_obs, nx, ny, rx,
                     ry, wx, wy, win, cells, sigma2, M);
}

int chol_max_order() { return kCholThreads; }

void launch_chol_factor(int n, double* A, int32_t* status, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(chol_factor_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * kCholThreads * kCholStride));
    attr = true;
  }
  hipLaunchKernelGGL(chol_factor_kernel, dim3(1), dim3(kCholThreads),
                     sizeof(double) * (size_t)n * kCholStride, s, n, A, status);
}

void launch_sd_full(int n, int ne, int stride, const double* S, const double* D, double* SD,
                    float* sdf, double* cval, hipStream_t s) {
  hipLaunchKernelGGL(sd_gemm_kernel, dim3((n + 15) / 16, (ne + 15) / 16), dim3(256), 0, s, n, ne,
                     stride, sd_float_stride(ne), S, D, SD, sdf);
  hipLaunchKernelGGL(dot_rows_kernel, dim3(ne), dim3(kThreads), 0, s, n, stride, D, SD, cval);
}

void launch_chol_solve(int n, int nrhs, const double* L, const double* rhs, int rhs_stride,
                       double* out, int out_stride, double* cval, hipStream_t s) {
  const int blocks = (nrhs + 3) / 4;
  if (n <= 512)
    hipLaunchKernelGGL(chol_solve_kernel<8>, dim3(blocks), dim3(256), 0, s, n, nrhs, L, rhs,
                       rhs_stride, out, out_stride, cval);
  else
    hipLaunchKernelGGL(chol_solve_kernel<16>, dim3(blocks), dim3(256), 0, s, n, nrhs, L, rhs,
                       rhs_stride, out, out_stride, cval);
}

void launch_observe(int n_obs, int nx, int ny, double H, double sigma, uint64_t seed,
                    uint64_t step, uint32_t ens, const float* truth, const int32_t* cells,
                    double* y, hipStream_t s) {
  hipLaunchKernelGGL(observe_kernel, dim3((n_obs + 127) / 128), dim3(128), 0, s, n_obs, nx, ny, H,
                     sigma, seed, step, ens, truth, cells, y);
}

void launch_cfl(int ne, int nx, int ny, float H, float g, const float* psi, unsigned* out,
                hipStream_t s) {
  const size_t total = (size_t)ne * nx * ny;
  size_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cfl_kernel, dim3((unsigned)blocks), dim3(256), 0, s, total, (size_t)nx * ny,
                     H, g, psi, out);
}

void launch_drift_k1(int ne, int nd, int nx, int ny, double dx, double dy, double H, double dt,
                     const float* psi, const double* pos, double* k1, double* pstar,
                     hipStream_t s, const float* psi_b, double w) {
  const int n = ne * nd;
  hipLaunchKernelGGL(drift_k1_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ne, nd, nx, ny, dx, dy,
                     H, dt, psi, psi_b ? psi_b : psi, psi_b ? w : 0.0, pos, k1, pstar);
}

void launch_drift_k2(int ne, int nd, int nx, int ny, double dx, double dy, double H, double dt,
                     const float* psi, double* pos, const double* k1, const double* pstar,
                     double* traj, hipStream_t s, const float* psi_b, double w) {
  const int n = ne * nd;
  hipLaunchKernelGGL(drift_k2_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ne, nd, nx, ny, dx, dy,
                     H, dt, psi, psi_b ? psi_b : psi, psi_b ? w : 0.0, pos, k1, pstar, traj);
}


void launch_gather_particles(int ne, size_t per_particle, const int32_t* parents, const float* in,
                             float* out, hipStream_t s) {
  const size_t n4 = per_particle / 4;
  size_t bx = (n4 + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)bx, ne), dim3(256), 0, s, n4, parents,
                     reinterpret_cast<const float4*>(in), reinterpret_cast<float4*>(out));
}

void launch_batch_stage_in(const BatchStageIn& a, int n, hipStream_t s) {
  hipLaunchKernelGGL(batch_stage_in_kernel, dim3(n), dim3(256), 0, s, a);
}

void launch_batch_status(const BatchStatusOut& a, int n, hipStream_t s) {
  hipLaunchKernelGGL(batch_status_kernel, dim3(1), dim3(64), 0, s, a, n);
}

void launch_resample(int ne, uint64_t seed, uint64_t step, uint32_t ens, const double* logw,
                     int32_t* parents, int32_t* counts, double* cum, hipStream_t s, double* scal) {
  hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(64), 0, s, ne, seed, step, ens, logw, parents,
                     counts, cum, scal);
}

}  // namespace iewpf
