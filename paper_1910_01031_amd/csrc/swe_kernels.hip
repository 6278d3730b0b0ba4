// Shallow-water scheme step (both SSP-RK2 stages fused) for gfx950.
//
// Scheme (Section "The simplified ocean model", eq. swe_full, eq. swecfl; the paper cites
// a well-balanced central-upwind scheme with a local Coriolis potential):
//   u = hu/h, v = hv/h;  x-faces reconstructed from K = g(eta - V) with the potential local
//   to each cell, V_{j+-1} = +-(f dx/2g)(v_j + v_{j+-1}); generalized-minmod slopes; face
//   eta = eta_j +- (sigma_K + f dx v_j)/(2g); y-faces symmetric with L = g(eta + U),
//   eta^{N,S} = eta_k +- (sigma_L - f dy u_k)/(2g); Kurganov-Petrova central-upwind
//   fluxes with momentum flux q u + g eta (H + eta/2); Coriolis source (f hv, -f hu);
//   psi* = psi + dt L(psi),  psi' = psi/2 + (psi* + dt L(psi*))/2.
//
// Mapping: one wave64 owns a strip of columns x0-4 .. x0+59 (lane = column) and marches
// down rows.  x-neighbours come from adjacent lanes (cross-lane moves), y-neighbours from
// registers holding the previous rows, so every cell's reconstruction and every face flux
// is computed once per stage.  Stage 1 runs two rows ahead of stage 2 inside the same
// wave; the intermediate psi* never leaves registers.  Each stage consumes two lanes per
// side, leaving 56 output columns per wave.  HBM traffic per scheme step: one read and
// one write of the state (24 B per cell) plus the strip halo rows.
#include <algorithm>
#include <type_traits>

#include "buffer_dev.hpp"
#include "internal.hpp"

namespace iewpf {
namespace {

// Cross-lane moves by one lane inside the wave64; lanes at the wave ends are never written
// back.  ds_bpermute is the default: the DPP wave shifts measured slower on gfx950.
#ifdef IEWPF_XLANE_DPP
__device__ __forceinline__ float lane_prev(float x) {  // value held by lane - 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138 /* wave_shr:1 */, 0xF,
                                                 0xF, true));
}
__device__ __forceinline__ float lane_next(float x) {  // value held by lane + 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130 /* wave_shl:1 */, 0xF,
                                                 0xF, true));
}
#else
__device__ __forceinline__ float lane_prev(float x) { return __shfl_up(x, 1, kWave); }
__device__ __forceinline__ float lane_next(float x) { return __shfl_down(x, 1, kWave); }
#endif

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrtf_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// Generalized minmod of (a, c, b) where c has the sign of a + b (c = (a + b) / (2 theta)):
// 0 unless a and b share a sign, else the one of the three nearest to 0, i.e.
// minmod(minmod(a, b), c) with minmod(x, y) = median(x, y, 0).  The result is one of the
// inputs or 0, so it is exact; two v_med3_f32.
__device__ __forceinline__ float minmod3(float a, float c, float b) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_fmed3f(a, b, 0.0f), c, 0.0f);
}

// The limiters below work on the slope divided by theta: minmod(theta a, c, theta b) =
// theta minmod(a, c / theta, b) for theta > 0, with the one-sided differences a, b and the
// central one c = (a + b) / 2, so only the central difference is scaled (by 1/(2 theta));
// theta goes into the constants that turn the slope into face offsets.

// Central-upwind flux between a left (-) and right (+) face state (eta, normal velocity,
// tangential velocity).  Outputs mass, normal-momentum and tangential-momentum fluxes.
__device__ __forceinline__ void cu_flux(float eL, float nL, float tL, float eR, float nR, float tR,
                                        const SweConst& C, float& F0, float& F1, float& F2) {
  const float hL = C.H + eL, hR = C.H + eR;
  const float qL = hL * nL, qR = hR * nR;
  const float cL = sqrtf_fast(C.g * hL), cR = sqrtf_fast(C.g * hR);
  const float ap = fmaxf(fmaxf(nL + cL, nR + cR), 0.0f);
  const float am = fminf(fminf(nL - cL, nR - cR), 0.0f);
  // F = wL F(-) - wR F(+) + apam (psi+ - psi-), wL = a+/(a+ - a-), wR = a-/(a+ - a-)
  const float inv = rcpf(ap - am);
  const float wL = ap * inv, wR = am * inv;
  const float apam = wL * am;
  const float wqL = wL * qL, wqR = wR * qR;
  // normal momentum flux q n + g eta (H + eta/2) = q n + eta (g H + (g/2) eta)
  const float gH = C.g * C.H, hg = 0.5f * C.g;
  const float ML = qL * nL + eL * (gH + hg * eL);
  const float MR = qR * nR + eR * (gH + hg * eR);
  F0 = (wqL - wqR) + apam * (eR - eL);
  F1 = wL * ML - wR * MR + apam * (qR - qL);
  // tangential momentum (p = h t): wL qL tL - wR qR tR + apam (pR - pL), grouped by side as
  // tL (wL qL - apam hL) - tR (wR qR - apam hR) (two multiplies and a subtraction fewer)
  const float bL = wqL - apam * hL, bR = wqR - apam * hR;
  F2 = tL * bL - tR * bR;
}

// x-direction flux divergence F_{j+1/2} - F_{j-1/2} of one row (mass, hu, hv).
__device__ __forceinline__ void x_divergence(float e, float u, float v, const SweConst& C,
                                             float& d0, float& d1, float& d2) {
  const float eE_ = lane_next(e), uE_ = lane_next(u), vE_ = lane_next(v);
  // Differences to the next cell, of K / g = eta - V / g (the potential in units of eta,
  // V / g = +-f dx (v + v_nb) / (2 g)), u and v.  The difference between cells j and j+1 is
  // the same whichever of the two the potential is local to, so the difference to the
  // previous cell is the previous lane's.
  const float bK = (eE_ - e) - C.fxg * (v + vE_);
  const float bu = uE_ - u, bv = vE_ - v;
  const float aK = lane_prev(bK), au = lane_prev(bu), av = lane_prev(bv);
  // slopes divided by theta: minmod(a, (a + b) / (2 theta), b)
  const float sK = minmod3(aK, (aK + bK) * C.k2t, bK);
  const float su = minmod3(au, (au + bu) * C.k2t, bu);
  const float sv = minmod3(av, (av + bv) * C.k2t, bv);
  // eta^{E,W} = eta +- (sigma_K + f dx v) / (2 g) = eta +- (theta sK / 2 + f dx v / (2 g));
  // u, v faces +- theta s / 2
  const float off = C.ht * sK + C.fxg * v;
  const float eEf = e + off, eWf = e - off;
  const float uEf = u + C.ht * su, uWf = u - C.ht * su;
  const float vEf = v + C.ht * sv, vWf = v - C.ht * sv;
  // face j+1/2: left = east face of this cell, right = west face of cell j+1
  float F0, F1, F2;
  cu_flux(eEf, uEf, vEf, lane_next(eWf), lane_next(uWf), lane_next(vWf), C, F0, F1, F2);
  d0 = F0 - lane_prev(F0);
  d1 = F1 - lane_prev(F1);  // x normal momentum = hu
  d2 = F2 - lane_prev(F2);  // x tangential momentum = hv
}

// y reconstruction of row k: north and south face states (eta, v = normal, u = tangential)
// from the differences to row k-1 (dLm, dum, dvm) and to row k+1 (dLp, dup, dvp), with
// L = g (eta + U) and U the Coriolis potential local to row k, carried as L / g.  The difference between rows
// k and k+1 is the same whichever of the two rows the potential is local to, so each one is
// computed once and serves both rows.
struct YFace {
  float e, n, t;
};
__device__ __forceinline__ void y_recon(float e, float u, float v, float dLm, float dum, float dvm,
                                        float dLp, float dup, float dvp, const SweConst& C,
                                        YFace& N, YFace& S) {
  // slopes divided by theta: minmod(a, (a + b) / (2 theta), b)
  const float sL = minmod3(dLm, (dLm + dLp) * C.k2t, dLp);
  const float su = minmod3(dum, (dum + dup) * C.k2t, dup);
  const float sv = minmod3(dvm, (dvm + dvp) * C.k2t, dvp);
  const float off = C.ht * sL - C.fyg * u;  // sL: slope of L / g divided by theta
  N.e = e + off;
  S.e = e - off;
  N.n = v + C.ht * sv;
  S.n = v - C.ht * sv;
  N.t = u + C.ht * su;
  S.t = u - C.ht * su;
}

// One RK stage as a row pipeline: push row m (eta, hu, hv), emit row m-2 of
// psi + dt L(psi) (the forward-Euler part of the stage).  The x divergence of row m-2 is
// computed when the row is emitted.  The mode skips what the rows at the top of a strip do
// not need:
//   kPushStore:    keep the row only;
//   kPushNoFlux:   y reconstruction of row m-1 only (the face above it is never used);
//   kPushFluxOnly: y reconstruction and y flux, nothing emitted (row m-2 is not needed);
//   kPushFull:     everything.
enum { kPushStore, kPushNoFlux, kPushFluxOnly, kPushFull };

struct StagePipe {
  // rows m-2 ("a") and m-1 ("b")
  float ea, qa, ra, ua, va;
  float eb, qb, rb, ub, vb;
  float dL, du, dv;  // y differences of L / g, u, v between rows m-1 and m-2 (potential local to either)
  YFace Na;          // north face state of row m-2
  float g0, g1, g2;  // y flux at face (m-2) - 1/2: mass, hv (normal), hu (tangential)

  template <int MODE>
  __device__ __forceinline__ void push(float e, float q, float r, const SweConst& C, float& oe,
                                       float& oq, float& orr) {
    const float rh = rcpf(C.H + e);
    const float u = q * rh, v = r * rh;
    const float dLn = (e - eb) + C.fyg * (ub + u);  // L / g, rows m and m-1
    const float dun = u - ub, dvn = v - vb;
    YFace Nb = {}, Sb = {};
    if (MODE != kPushStore) y_recon(eb, ub, vb, dL, du, dv, dLn, dun, dvn, C, Nb, Sb);  // row m-1
    float G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;                                     // face (m-2) + 1/2
    if (MODE == kPushFluxOnly || MODE == kPushFull)
      cu_flux(Na.e, Na.n, Na.t, Sb.e, Sb.n, Sb.t, C, G0, G1, G2);
    if (MODE == kPushFull) {
      float x0, x1, x2;
      x_divergence(ea, ua, va, C, x0, x1, x2);  // row m-2
      // psi + dt L(psi) with dt/dx, dt/dy and dt f as constants (one fused multiply-add per
      // term)
      oe = ea - C.dtidx * x0 - C.dtidy * (G0 - g0);
      oq = qa + C.dtf * ra - C.dtidx * x1 - C.dtidy * (G2 - g2);
      orr = ra - C.dtf * qa - C.dtidx * x2 - C.dtidy * (G1 - g1);
    } else {
      oe = oq = orr = 0.0f;
    }
    // advance
    ea = eb; qa = qb; ra = rb; ua = ub; va = vb;
    eb = e; qb = q; rb = r; ub = u; vb = v;
    dL = dLn; du = dun; dv = dvn;
    Na = Nb;
    g0 = G0; g1 = G1; g2 = G2;
  }
};

template <int V>
using PushMode = std::integral_constant<int, V>;

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}
// i in [-n, 2n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// One particle's [3][ny][nx] state as a raw buffer: the field and row go into the scalar
// offset, the lane's column into one VGPR set up once per wave.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const float* base, size_t ncell) {
  return make_rsrc(base, 12 * ncell);
}

__device__ __forceinline__ void cr_weights(float t, float w[4]) {
  const float t2 = t * t, t3 = t2 * t;
  w[0] = 0.5f * (-t3 + 2.0f * t2 - t);
  w[1] = 0.5f * (3.0f * t3 - 5.0f * t2 + 2.0f);
  w[2] = 0.5f * (-3.0f * t3 + 4.0f * t2 + t);
  w[3] = 0.5f * (t3 - t2);
}

// Model-error interpolation I_Omega of the coarse field z down the rows of a strip.  Each
// lane keeps the x-interpolated values of the four coarse rows around the current fine
// row; the window advances by one coarse row every c fine rows (the only loads), and a
// fine row costs one 4-tap interpolation in y.  Coarse point b sits at (b + 1/2) c dy.
// The four coarse values of the row that enters next are loaded one window step ahead, so
// their latency is hidden behind c fine rows.
struct CoarseRows {
  int cx[4];
  float wx[4];
  float xr[4];   // x-interpolated coarse rows by-1 .. by+2
  float nr[4];   // raw values of coarse row by+3 (prefetched)
  int by;        // base coarse row of the current window

  __device__ __forceinline__ float combine(const float r[4]) const {
    return wx[0] * r[0] + wx[1] * r[1] + wx[2] * r[2] + wx[3] * r[3];
  }
  __device__ __forceinline__ void fetch(const float* __restrict__ z, const SweConst& C, int b,
                                        float r[4]) const {
    const float* row = z + (size_t)wrap1(b, C.nry) * C.nrx;
#pragma unroll
    for (int m = 0; m < 4; ++m) r[m] = row[cx[m]];
  }
  __device__ __forceinline__ float xrow(const float* __restrict__ z, const SweConst& C, int b) const {
    float r[4];
    fetch(z, C, b, r);
    return combine(r);
  }
  __device__ __forceinline__ void init(const float* __restrict__ z, const SweConst& C, int jw,
                                       int s) {
    const int num = 2 * jw + 1 - C.c;
    const int bx = (num >= 0 ? num : num - 2 * C.c + 1) / (2 * C.c);
    cr_weights(static_cast<float>(num - 2 * C.c * bx) / static_cast<float>(2 * C.c), wx);
#pragma unroll
    for (int m = 0; m < 4; ++m) cx[m] = wrap1(bx + m - 1, C.nrx);
    const int ns = 2 * s + 1 - C.c;
    by = (ns >= 0 ? ns : ns - 2 * C.c + 1) / (2 * C.c);
#pragma unroll
    for (int n = 0; n < 4; ++n) xr[n] = xrow(z, C, by + n - 1);
    fetch(z, C, by + 3, nr);
  }
  // value at fine row s (unwrapped, non-decreasing between calls, s - previous s <= c)
  __device__ __forceinline__ float at(const float* __restrict__ z, const SweConst& C, int s) {
    const int ns = 2 * s + 1 - C.c;
    const int b = (ns >= 0 ? ns : ns - 2 * C.c + 1) / (2 * C.c);
    if (b != by) {  // wave-uniform: advance the window by one coarse row
      xr[0] = xr[1];
      xr[1] = xr[2];
      xr[2] = xr[3];
      xr[3] = combine(nr);  // row b + 2 = old by + 3
      by = b;
      fetch(z, C, b + 3, nr);
    }
    const int ph = ns - 2 * C.c * b;  // wave-uniform phase of the row, in [0, 2c)
    float wy[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) wy[n] = C.cr.w[ph][n];
    return wy[0] * xr[0] + wy[1] * xr[1] + wy[2] * xr[2] + wy[3] * xr[3];
  }
};

// One scheme step of every particle.  NOISE: also add the model error Q_GB I_Omega z to the
// output (z = SOAR xi on the coarse grid, one [nry][nrx] field per particle).
#ifndef IEWPF_SWE_MIN_BLOCKS
#define IEWPF_SWE_MIN_BLOCKS 1
#endif

#ifndef IEWPF_SWE_PREFETCH
#define IEWPF_SWE_PREFETCH 3
#endif
static_assert(IEWPF_SWE_PREFETCH >= 1 && IEWPF_SWE_PREFETCH <= 8, "prefetch distance");

template <bool NOISE>
__device__ __forceinline__ void substep_wave(const float* __restrict__ in, float* __restrict__ out,
                                             const float* __restrict__ zall, const SweConst& C,
                                             int wave) {
  const int lane = threadIdx.x & (kWave - 1);
  const int per_particle = C.n_strip_x * C.n_strip_y;
  const int particle = wave / per_particle;
  const int rem = wave - particle * per_particle;
  const int sy = rem / C.n_strip_x;
  const int sx = rem - sy * C.n_strip_x;
  const int nx = C.nx, ny = C.ny;
  const size_t ncell = (size_t)nx * ny;
  // byte offsets below 12 nx ny < 2^31 (checked when the context is created)
  const __amdgpu_buffer_rsrc_t bin = state_rsrc(in + (size_t)particle * 3 * ncell, ncell);
  const __amdgpu_buffer_rsrc_t bout = state_rsrc(out + (size_t)particle * 3 * ncell, ncell);
  const unsigned fq = 4u * static_cast<unsigned>(ncell), fr = 2u * fq;  // field byte offsets
  const unsigned brow = 4u * static_cast<unsigned>(nx);                  // row stride in bytes

  const int j = sx * kSweOut + lane - kSweHalo;  // unwrapped column
  const int jw = wrap(j, nx);
  const bool writer = lane >= kSweHalo && lane < kWave - kSweHalo && j < nx;
  const unsigned bjw = 4u * static_cast<unsigned>(jw);  // byte offset of the lane's column
  // With model error, lanes that write nothing get an offset past the buffer (their stores
  // are dropped), so the row store needs no branch; the plain step keeps the branch, which
  // measured faster there (the branch-free form let the scheduler raise register use).
  const unsigned bj = (NOISE && !writer) ? kBufferOff : 4u * static_cast<unsigned>(j);
  const int k0 = sy * C.strip_h;
  const int k_end = min(k0 + C.strip_h, ny);  // exclusive

  const float* z = nullptr;
  CoarseRows cr;
  if (NOISE) {
    z = zall + (size_t)particle * C.nrx * C.nry;
    cr.init(z, C, jw, k0 - 1);  // first model-error row needed: k0 - 1
  }

  StagePipe s1 = {}, s2 = {};
  // psi^n rows m-4 .. m-1 (before the push of row m) for the stage-2 combination
  float pe4 = 0, pq4 = 0, pr4 = 0, pe3 = 0, pq3 = 0, pr3 = 0, pe2 = 0, pq2 = 0, pr2 = 0;
  float pe1 = 0, pq1 = 0, pr1 = 0;
  float dA = 0.0f, dB = 0.0f;  // model-error d_eta rows m-5, m-4

  // rows m .. m + kPf - 1 are loaded (in flight) before row m is pushed
  constexpr int kPf = IEWPF_SWE_PREFETCH;
  float ne_[kPf], nq_[kPf], nr_[kPf];
#pragma unroll
  for (int i = 0; i < kPf; ++i) {
    const unsigned off = static_cast<unsigned>(wrap(k0 - 4 + i, ny)) * brow;
    ne_[i] = ld_buf(bin, bjw, off);
    nq_[i] = ld_buf(bin, bjw, off + fq);
    nr_[i] = ld_buf(bin, bjw, off + fr);
  }

  // Rows m = k0-4 .. k0-1: stage 1 only; k0 .. k0+3: both stages, no output yet;
  // k0+4 .. k_end+3: both stages and row m-4 written.  Stage 1 must produce rows
  // k0-2 .. k_end+1 and stage 2 rows k0 .. k_end-1; the push modes drop the rows above.
  auto step = [&](int m, auto mode1, auto mode2, bool emit) {
    constexpr int M1 = decltype(mode1)::value, M2 = decltype(mode2)::value;
    constexpr bool stage2 = M2 >= 0;
    const float e = ne_[0], q = nq_[0], r = nr_[0];
#pragma unroll
    for (int i = 0; i + 1 < kPf; ++i) {
      ne_[i] = ne_[i + 1];
      nq_[i] = nq_[i + 1];
      nr_[i] = nr_[i + 1];
    }
    // m + kPf < ny + 3 + kPf < 3 ny (ny >= 7): two conditional wraps suffice
    const unsigned o2 = static_cast<unsigned>(wrap1(wrap1(m + kPf, ny), ny)) * brow;
    ne_[kPf - 1] = ld_buf(bin, bjw, o2);
    nq_[kPf - 1] = ld_buf(bin, bjw, o2 + fq);
    nr_[kPf - 1] = ld_buf(bin, bjw, o2 + fr);
    float se, sq, sr;
    s1.template push<M1>(e, q, r, C, se, sq, sr);  // psi* of row m - 2
    const float qe4 = pe4, qq4 = pq4, qr4 = pr4;
    pe4 = pe3; pq4 = pq3; pr4 = pr3;
    pe3 = pe2; pq3 = pq2; pr3 = pr2;
    pe2 = pe1; pq2 = pq1; pr2 = pr1;
    pe1 = e; pq1 = q; pr1 = r;
    float dC = 0.0f;
    // d_eta row m-3, needed from m = k0 + 2 on (row k0 - 1), the first row pushed into
    // stage 2 with a mode other than Store: a compile-time test instead of a run-time one
    if (NOISE && M2 > kPushStore) dC = cr.at(z, C, m - 3);
    if (stage2) {
      float te, tq, tr;
      s2.template push<(M2 < 0 ? kPushStore : M2)>(se, sq, sr, C, te, tq, tr);  // row m - 4
      if (emit) {
        float oe = 0.5f * (qe4 + te), oq = 0.5f * (qq4 + tq), orr = 0.5f * (qr4 + tr);
        if (NOISE) {
          oe += dB;
          oq += -C.gb_y * (dC - dA);
          orr += C.gb_x * (lane_next(dB) - lane_prev(dB));
        }
        if (NOISE || writer) {
          const unsigned o = static_cast<unsigned>(m - 4) * brow;
          st_buf(bout, bj, o, oe);
          st_buf(bout, bj, o + fq, oq);
          st_buf(bout, bj, o + fr, orr);
        }
      }
    }
    if (NOISE) {
      dA = dB;
      dB = dC;
    }
  };
  using Off = PushMode<-1>;
  using Store = PushMode<kPushStore>;
  using NoFlux = PushMode<kPushNoFlux>;
  using FluxOnly = PushMode<kPushFluxOnly>;
  using Full = PushMode<kPushFull>;
  step(k0 - 4, Store{}, Off{}, false);
  step(k0 - 3, Store{}, Off{}, false);
  step(k0 - 2, NoFlux{}, Off{}, false);
  step(k0 - 1, FluxOnly{}, Off{}, false);
  step(k0, Full{}, Store{}, false);
  step(k0 + 1, Full{}, Store{}, false);
  step(k0 + 2, Full{}, NoFlux{}, false);
  step(k0 + 3, Full{}, FluxOnly{}, false);
  // eight rows per trip (a multiple of the period of the row rotation, so the pipeline
  // registers are renamed instead of moved; the loop head's waits for loads in flight come
  // once per eight rows), then four, then single rows
  int m = k0 + 4;
  for (; m + 7 <= k_end + 3; m += 8) {
    step(m, Full{}, Full{}, true);
    step(m + 1, Full{}, Full{}, true);
    step(m + 2, Full{}, Full{}, true);
    step(m + 3, Full{}, Full{}, true);
    step(m + 4, Full{}, Full{}, true);
    step(m + 5, Full{}, Full{}, true);
    step(m + 6, Full{}, Full{}, true);
    step(m + 7, Full{}, Full{}, true);
  }
  for (; m + 3 <= k_end + 3; m += 4) {
    step(m, Full{}, Full{}, true);
    step(m + 1, Full{}, Full{}, true);
    step(m + 2, Full{}, Full{}, true);
    step(m + 3, Full{}, Full{}, true);
  }
  for (; m <= k_end + 3; ++m) step(m, Full{}, Full{}, true);
}

// MASKED: particles i with mask[i] == 0 are not stepped (their waves return at once)
template <bool NOISE, bool MASKED = false>
__global__ __launch_bounds__(256, IEWPF_SWE_MIN_BLOCKS) void swe_substep_kernel(
    const float* __restrict__ in, float* __restrict__ out, const float* __restrict__ zall,
    SweConst C, int total_waves, const int32_t* __restrict__ mask) {
  // wave-uniform: held in scalar registers, so the strip and particle offsets are scalar
  const int wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave));
  if (wave >= total_waves) return;  // whole wave exits together
  if (MASKED && mask[wave / (C.n_strip_x * C.n_strip_y)] == 0) return;
  substep_wave<NOISE>(in, out, zall, C, wave);
}

// Several ensembles of different grids in one launch: the waves of ensemble e are
// [job[e].wave_begin, job[e+1].wave_begin); parity selects which of the two buffers of
// every ensemble is the input.  With NOISE every job's z is set (the host builds the two
// tables that way).
template <bool NOISE>
__global__ __launch_bounds__(256, IEWPF_SWE_MIN_BLOCKS) void swe_batch_kernel(
    const SweJobTable* __restrict__ tab, int parity, int zstep) {
  const int wave =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave));
  if (wave >= tab->total_waves) return;
  int e = 0;
  while (e + 1 < tab->n && wave >= tab->job[e + 1].wave_begin) ++e;
  const SweJob& J = tab->job[e];
  const float* in = parity ? J.buf_b : J.buf_a;
  float* out = parity ? J.buf_a : J.buf_b;
  // with NOISE, the field of model step zstep of the chunk drawn ahead
  substep_wave<NOISE>(in, out, NOISE ? J.z + (size_t)zstep * J.z_field : nullptr, J.C,
                      wave - J.wave_begin);
}

// ---- full-row form: one workgroup of W = ceil(nx / 64) waves owns whole rows ------------
// Thread t of the workgroup is column t (t < nx), so the periodic row needs no halo columns
// and no column is computed twice.  The x-neighbours travel through LDS; the x passes of the
// two RK stages (stage 1 on psi row m-2, stage 2 on psi* row m-4) are independent within a
// step, so they share each exchange: three exchanges and three barriers per row.  The
// arithmetic is the strip form's, term for term (the difference to the previous cell is
// formed from the exchanged values exactly as the neighbour forms its own), so the results
// are bit-identical to it.

// One RK stage with the push split around the x pass: ypart() takes the new row (primitive
// variables, y reconstruction of row m-1, y flux at face (m-2)+1/2); finish() applies the x
// divergence of row m-2 and advances the rows.
struct RowStage {
  float ea, qa, ra, ua, va;
  float eb, qb, rb, ub, vb;
  float dL, du, dv;
  YFace Na;
  float g0, g1, g2;
  float un, vn, dLn, dun, dvn;  // of the row being pushed
  YFace Nb;
  float G0, G1, G2;

  template <int MODE>
  __device__ __forceinline__ void ypart(float e, float q, float r, const SweConst& C) {
    const float rh = rcpf(C.H + e);
    un = q * rh;
    vn = r * rh;
    dLn = (e - eb) + C.fyg * (ub + un);
    dun = un - ub;
    dvn = vn - vb;
    YFace Sb = {};
    Nb = {};
    if (MODE != kPushStore) y_recon(eb, ub, vb, dL, du, dv, dLn, dun, dvn, C, Nb, Sb);
    G0 = G1 = G2 = 0.0f;
    if (MODE == kPushFluxOnly || MODE == kPushFull)
      cu_flux(Na.e, Na.n, Na.t, Sb.e, Sb.n, Sb.t, C, G0, G1, G2);
  }
  template <int MODE>
  __device__ __forceinline__ void finish(float e, float q, float r, float x0, float x1, float x2,
                                         const SweConst& C, float& oe, float& oq, float& orr) {
    if (MODE == kPushFull) {
      oe = ea - C.dtidx * x0 - C.dtidy * (G0 - g0);
      oq = qa + C.dtf * ra - C.dtidx * x1 - C.dtidy * (G2 - g2);
      orr = ra - C.dtf * qa - C.dtidx * x2 - C.dtidy * (G1 - g1);
    } else {
      oe = oq = orr = 0.0f;
    }
    ea = eb; qa = qb; ra = rb; ua = ub; va = vb;
    eb = e; qb = q; rb = r; ub = un; vb = vn;
    dL = dLn; du = dun; dv = dvn;
    Na = Nb;
    g0 = G0; g1 = G1; g2 = G2;
  }
};

// Face states of a row from its own values and its two x-neighbours' (x_divergence's
// reconstruction with the neighbour lanes' values supplied).
struct XFaces {
  float eE, uE, vE, eW, uW, vW;
};
__device__ __forceinline__ XFaces x_faces(float e, float u, float v, float eE_, float uE_, float vE_,
                                          float eW_, float uW_, float vW_, const SweConst& C) {
  const float bK = (eE_ - e) - C.fxg * (v + vE_);
  const float bu = uE_ - u, bv = vE_ - v;
  // the previous cell's differences to this one, formed as that cell forms them
  const float aK = (e - eW_) - C.fxg * (vW_ + v);
  const float au = u - uW_, av = v - vW_;
  const float sK = minmod3(aK, (aK + bK) * C.k2t, bK);
  const float su = minmod3(au, (au + bu) * C.k2t, bu);
  const float sv = minmod3(av, (av + bv) * C.k2t, bv);
  const float off = C.ht * sK + C.fxg * v;
  XFaces F;
  F.eE = e + off;
  F.eW = e - off;
  F.uE = u + C.ht * su;
  F.uW = u - C.ht * su;
  F.vE = v + C.ht * sv;
  F.vW = v - C.ht * sv;
  return F;
}

template <bool NOISE, int STRIDE>
__device__ __forceinline__ void row_strip(const float* __restrict__ in, float* __restrict__ out,
                                          const float* __restrict__ zall, const SweConst& C,
                                          int particle, int sy, float* __restrict__ xl) {
  const int j = threadIdx.x;
  const int nx = C.nx, ny = C.ny;
  const size_t ncell = (size_t)nx * ny;
  const bool active = j < nx;
  // neighbour columns on the torus (an idle thread past the row reads its own slot)
  const int jn = !active ? j : (j + 1 == nx ? 0 : j + 1);
  const int jp = !active ? j : (j == 0 ? nx - 1 : j - 1);
  const __amdgpu_buffer_rsrc_t bin = state_rsrc(in + (size_t)particle * 3 * ncell, ncell);
  const __amdgpu_buffer_rsrc_t bout = state_rsrc(out + (size_t)particle * 3 * ncell, ncell);
  const unsigned fq = 4u * static_cast<unsigned>(ncell), fr = 2u * fq;
  const unsigned brow = 4u * static_cast<unsigned>(nx);
  // idle threads read zeros and write nothing
  const unsigned bj = active ? 4u * static_cast<unsigned>(j) : kBufferOff;
  const int k0 = sy * C.strip_h;
  const int k_end = min(k0 + C.strip_h, ny);

  const float* z = nullptr;
  CoarseRows cr;
  if (NOISE) {
    z = zall + (size_t)particle * C.nrx * C.nry;
    cr.init(z, C, active ? j : j % nx, k0 - 1);
  }
  // LDS: three regions (one per exchange of a row) of 7 quantities x STRIDE columns
  auto slot = [&](int region, int qn) { return xl + (region * 7 + qn) * STRIDE; };

  RowStage s1 = {}, s2 = {};
  float pe4 = 0, pq4 = 0, pr4 = 0, pe3 = 0, pq3 = 0, pr3 = 0, pe2 = 0, pq2 = 0, pr2 = 0;
  float pe1 = 0, pq1 = 0, pr1 = 0;
  float dA = 0.0f, dB = 0.0f;

  constexpr int kPf = IEWPF_SWE_PREFETCH;
  float ne_[kPf], nq_[kPf], nr_[kPf];
#pragma unroll
  for (int i = 0; i < kPf; ++i) {
    const unsigned off = static_cast<unsigned>(wrap(k0 - 4 + i, ny)) * brow;
    ne_[i] = ld_buf(bin, bj, off);
    nq_[i] = ld_buf(bin, bj, off + fq);
    nr_[i] = ld_buf(bin, bj, off + fr);
  }

  auto step = [&](int m, auto mode1, auto mode2, bool emit) {
    constexpr int M1 = decltype(mode1)::value, M2 = decltype(mode2)::value;
    constexpr bool stage2 = M2 >= 0;
    constexpr bool x1 = M1 == kPushFull, x2 = M2 == kPushFull;
    const float e = ne_[0], q = nq_[0], r = nr_[0];
#pragma unroll
    for (int i = 0; i + 1 < kPf; ++i) {
      ne_[i] = ne_[i + 1];
      nq_[i] = nq_[i + 1];
      nr_[i] = nr_[i + 1];
    }
    const unsigned o2 = static_cast<unsigned>(wrap1(wrap1(m + kPf, ny), ny)) * brow;
    ne_[kPf - 1] = ld_buf(bin, bj, o2);
    nq_[kPf - 1] = ld_buf(bin, bj, o2 + fq);
    nr_[kPf - 1] = ld_buf(bin, bj, o2 + fr);
    s1.template ypart<M1>(e, q, r, C);
    // x passes: stage 1 on its row m-2, stage 2 on its row m-4 (both rows pushed earlier)
    float a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0, dBn = 0, dBp = 0;
    if (x1 || x2) {
      float* R0 = slot(0, 0);
      if (x1) {
        R0[j] = s1.ea;
        R0[STRIDE + j] = s1.ua;
        R0[2 * STRIDE + j] = s1.va;
      }
      if (x2) {
        R0[3 * STRIDE + j] = s2.ea;
        R0[4 * STRIDE + j] = s2.ua;
        R0[5 * STRIDE + j] = s2.va;
      }
      if (NOISE && x2) R0[6 * STRIDE + j] = dB;
      __syncthreads();
      XFaces f1 = {}, f2 = {};
      if (x1)
        f1 = x_faces(s1.ea, s1.ua, s1.va, R0[jn], R0[STRIDE + jn], R0[2 * STRIDE + jn], R0[jp],
                     R0[STRIDE + jp], R0[2 * STRIDE + jp], C);
      if (x2)
        f2 = x_faces(s2.ea, s2.ua, s2.va, R0[3 * STRIDE + jn], R0[4 * STRIDE + jn],
                     R0[5 * STRIDE + jn], R0[3 * STRIDE + jp], R0[4 * STRIDE + jp],
                     R0[5 * STRIDE + jp], C);
      if (NOISE && x2) {
        dBn = R0[6 * STRIDE + jn];
        dBp = R0[6 * STRIDE + jp];
      }
      float* R1 = slot(1, 0);
      if (x1) {
        R1[j] = f1.eW;
        R1[STRIDE + j] = f1.uW;
        R1[2 * STRIDE + j] = f1.vW;
      }
      if (x2) {
        R1[3 * STRIDE + j] = f2.eW;
        R1[4 * STRIDE + j] = f2.uW;
        R1[5 * STRIDE + j] = f2.vW;
      }
      __syncthreads();
      float F10 = 0, F11 = 0, F12 = 0, F20 = 0, F21 = 0, F22 = 0;
      if (x1)
        cu_flux(f1.eE, f1.uE, f1.vE, R1[jn], R1[STRIDE + jn], R1[2 * STRIDE + jn], C, F10, F11, F12);
      if (x2)
        cu_flux(f2.eE, f2.uE, f2.vE, R1[3 * STRIDE + jn], R1[4 * STRIDE + jn], R1[5 * STRIDE + jn],
                C, F20, F21, F22);
      float* R2 = slot(2, 0);
      if (x1) {
        R2[j] = F10;
        R2[STRIDE + j] = F11;
        R2[2 * STRIDE + j] = F12;
      }
      if (x2) {
        R2[3 * STRIDE + j] = F20;
        R2[4 * STRIDE + j] = F21;
        R2[5 * STRIDE + j] = F22;
      }
      __syncthreads();
      if (x1) {
        a0 = F10 - R2[jp];
        a1 = F11 - R2[STRIDE + jp];
        a2 = F12 - R2[2 * STRIDE + jp];
      }
      if (x2) {
        b0 = F20 - R2[3 * STRIDE + jp];
        b1 = F21 - R2[4 * STRIDE + jp];
        b2 = F22 - R2[5 * STRIDE + jp];
      }
    }
    float se, sq, sr;
    s1.template finish<M1>(e, q, r, a0, a1, a2, C, se, sq, sr);  // psi* of row m - 2
    const float qe4 = pe4, qq4 = pq4, qr4 = pr4;
    pe4 = pe3; pq4 = pq3; pr4 = pr3;
    pe3 = pe2; pq3 = pq2; pr3 = pr2;
    pe2 = pe1; pq2 = pq1; pr2 = pr1;
    pe1 = e; pq1 = q; pr1 = r;
    float dC = 0.0f;
    if (NOISE && M2 > kPushStore) dC = cr.at(z, C, m - 3);
    if (stage2) {
      constexpr int M2s = M2 < 0 ? kPushStore : M2;
      float te, tq, tr;
      s2.template ypart<M2s>(se, sq, sr, C);
      s2.template finish<M2s>(se, sq, sr, b0, b1, b2, C, te, tq, tr);  // row m - 4
      if (emit) {
        float oe = 0.5f * (qe4 + te), oq = 0.5f * (qq4 + tq), orr = 0.5f * (qr4 + tr);
        if (NOISE) {
          oe += dB;
          oq += -C.gb_y * (dC - dA);
          orr += C.gb_x * (dBn - dBp);
        }
        const unsigned o = static_cast<unsigned>(m - 4) * brow;
        st_buf(bout, bj, o, oe);
        st_buf(bout, bj, o + fq, oq);
        st_buf(bout, bj, o + fr, orr);
      }
    }
    if (NOISE) {
      dA = dB;
      dB = dC;
    }
  };
  using Off = PushMode<-1>;
  using Store = PushMode<kPushStore>;
  using NoFlux = PushMode<kPushNoFlux>;
  using FluxOnly = PushMode<kPushFluxOnly>;
  using Full = PushMode<kPushFull>;
  step(k0 - 4, Store{}, Off{}, false);
  step(k0 - 3, Store{}, Off{}, false);
  step(k0 - 2, NoFlux{}, Off{}, false);
  step(k0 - 1, FluxOnly{}, Off{}, false);
  step(k0, Full{}, Store{}, false);
  step(k0 + 1, Full{}, Store{}, false);
  step(k0 + 2, Full{}, NoFlux{}, false);
  step(k0 + 3, Full{}, FluxOnly{}, false);
  int m = k0 + 4;
  for (; m + 7 <= k_end + 3; m += 8) {
    step(m, Full{}, Full{}, true);
    step(m + 1, Full{}, Full{}, true);
    step(m + 2, Full{}, Full{}, true);
    step(m + 3, Full{}, Full{}, true);
    step(m + 4, Full{}, Full{}, true);
    step(m + 5, Full{}, Full{}, true);
    step(m + 6, Full{}, Full{}, true);
    step(m + 7, Full{}, Full{}, true);
  }
  for (; m + 3 <= k_end + 3; m += 4) {
    step(m, Full{}, Full{}, true);
    step(m + 1, Full{}, Full{}, true);
    step(m + 2, Full{}, Full{}, true);
    step(m + 3, Full{}, Full{}, true);
  }
  for (; m <= k_end + 3; ++m) step(m, Full{}, Full{}, true);
}

#ifndef IEWPF_ROW_MIN_WAVES
#define IEWPF_ROW_MIN_WAVES 4
#endif

// grid: n_particles x n_strip_y workgroups of W x 64 threads (W x 64 <= STRIDE); MASKED:
// particles i with mask[i] == 0 are not stepped (their workgroups return at once)
template <bool NOISE, int STRIDE, bool MASKED = false>
__global__ __launch_bounds__(STRIDE, IEWPF_ROW_MIN_WAVES) void swe_row_kernel(
    const float* __restrict__ in, float* __restrict__ out, const float* __restrict__ zall,
    SweConst C, const int32_t* __restrict__ mask) {
  __shared__ float xl[3 * 7 * STRIDE];
  const int b = blockIdx.x;
  const int particle = b / C.n_strip_y;
  const int sy = b - particle * C.n_strip_y;
  if (MASKED && mask[particle] == 0) return;  // the whole workgroup
  row_strip<NOISE, STRIDE>(in, out, zall, C, particle, sy, xl);
}

template <int STRIDE>
void launch_row(const SweConst& C, int ne, const float* in, float* out, const float* z,
                hipStream_t s, const int32_t* mask) {
  const int threads = ((C.nx + 63) / 64) * 64;
  const int blocks = ne * C.n_strip_y;
  if (z)
    hipLaunchKernelGGL((swe_row_kernel<true, STRIDE>), dim3(blocks), dim3(threads), 0, s, in, out, z, C,
                       nullptr);
  else if (mask)  // masked steps are plain steps (the fallback of the surrogate window)
    hipLaunchKernelGGL((swe_row_kernel<false, STRIDE, true>), dim3(blocks), dim3(threads), 0, s, in,
                       out, z, C, mask);
  else
    hipLaunchKernelGGL((swe_row_kernel<false, STRIDE>), dim3(blocks), dim3(threads), 0, s, in, out, z,
                       C, nullptr);
}

}  // namespace

int swe_waves_per_cu() {
  int a = 0, b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, swe_substep_kernel<true>, 256, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, swe_substep_kernel<false>, 256, 0) != hipSuccess)
    return 16;
  return 4 * std::max(1, std::min(a, b));
}

int swe_row_blocks_per_cu(int nx) {
  const int threads = ((nx + 63) / 64) * 64;
  int a = 0, b = 0;
  hipError_t e1, e2;
  if (nx <= 256) {
    e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, swe_row_kernel<true, 256>, threads, 0);
    e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, swe_row_kernel<false, 256>, threads, 0);
  } else {
    e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, swe_row_kernel<true, 512>, threads, 0);
    e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, swe_row_kernel<false, 512>, threads, 0);
  }
  if (e1 != hipSuccess || e2 != hipSuccess) return 1;
  return std::max(1, std::min(a, b));
}

void launch_swe_batch(const SweJobTable* tab, int total_waves, int parity, bool noise, int zstep,
                      hipStream_t s) {
  const int blocks = (total_waves + 3) / 4;
  if (noise)
    hipLaunchKernelGGL(swe_batch_kernel<true>, dim3(blocks), dim3(256), 0, s, tab, parity, zstep);
  else
    hipLaunchKernelGGL(swe_batch_kernel<false>, dim3(blocks), dim3(256), 0, s, tab, parity, 0);
}

void launch_swe_substep(const SweConst& C, int ne, const float* in, float* out, const float* z,
                        hipStream_t s, const int32_t* mask) {
  if (C.row) {  // full-row form (nx <= 512)
    if (C.nx <= 256)
      launch_row<256>(C, ne, in, out, z, s, mask);
    else
      launch_row<512>(C, ne, in, out, z, s, mask);
    return;
  }
  const int total = ne * C.n_strip_x * C.n_strip_y;
  const int blocks = (total + 3) / 4;
  if (z)
    hipLaunchKernelGGL(swe_substep_kernel<true>, dim3(blocks), dim3(256), 0, s, in, out, z, C, total,
                       nullptr);
  else if (mask)
    hipLaunchKernelGGL((swe_substep_kernel<false, true>), dim3(blocks), dim3(256), 0, s, in, out, z,
                       C, total, mask);
  else
    hipLaunchKernelGGL(swe_substep_kernel<false>, dim3(blocks), dim3(256), 0, s, in, out, z, C,
                       total, nullptr);
}

}  // namespace iewpf
