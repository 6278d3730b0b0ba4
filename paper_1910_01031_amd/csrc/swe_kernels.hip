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
#include "internal.hpp"

namespace iewpf {
namespace {

__device__ __forceinline__ float lane_prev(float x) {  // value held by lane - 1
  return __shfl_up(x, 1, kWave);
}
__device__ __forceinline__ float lane_next(float x) {  // value held by lane + 1
  return __shfl_down(x, 1, kWave);
}

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrtf_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// Generalized minmod of three slopes.
__device__ __forceinline__ float minmod3(float a, float b, float c) {
  const float lo = fminf(a, fminf(b, c));
  const float hi = fmaxf(a, fmaxf(b, c));
  return lo > 0.0f ? lo : (hi < 0.0f ? hi : 0.0f);
}

__device__ __forceinline__ float limited(float qm, float q0, float qp, float theta) {
  return minmod3(theta * (q0 - qm), 0.5f * (qp - qm), theta * (qp - q0));
}

// Central-upwind flux between a left (-) and right (+) face state (eta, normal velocity,
// tangential velocity).  Outputs mass, normal-momentum and tangential-momentum fluxes.
__device__ __forceinline__ void cu_flux(float eL, float nL, float tL, float eR, float nR, float tR,
                                        const SweConst& C, float& F0, float& F1, float& F2) {
  const float hL = C.H + eL, hR = C.H + eR;
  const float qL = hL * nL, qR = hR * nR;
  const float pL = hL * tL, pR = hR * tR;
  const float cL = sqrtf_fast(C.g * hL), cR = sqrtf_fast(C.g * hR);
  const float ap = fmaxf(fmaxf(nL + cL, nR + cR), 0.0f);
  const float am = fminf(fminf(nL - cL, nR - cR), 0.0f);
  const float inv = rcpf(ap - am);
  const float apam = ap * am * inv;
  const float ML = qL * nL + C.g * eL * (C.H + 0.5f * eL);
  const float MR = qR * nR + C.g * eR * (C.H + 0.5f * eR);
  F0 = (ap * qL - am * qR) * inv + apam * (eR - eL);
  F1 = (ap * ML - am * MR) * inv + apam * (qR - qL);
  F2 = (ap * (qL * tL) - am * (qR * tR)) * inv + apam * (pR - pL);
}

// x-direction flux divergence F_{j+1/2} - F_{j-1/2} of one row (mass, hu, hv).
__device__ __forceinline__ void x_divergence(float e, float u, float v, const SweConst& C,
                                             float& d0, float& d1, float& d2) {
  const float eW_ = lane_prev(e), eE_ = lane_next(e);
  const float uW_ = lane_prev(u), uE_ = lane_next(u);
  const float vW_ = lane_prev(v), vE_ = lane_next(v);
  const float Kc = C.g * e;
  const float Kp = C.g * eE_ - C.hfdx * (v + vE_);
  const float Km = C.g * eW_ + C.hfdx * (v + vW_);
  const float sK = limited(Km, Kc, Kp, C.theta);
  const float su = limited(uW_, u, uE_, C.theta);
  const float sv = limited(vW_, v, vE_, C.theta);
  const float off = (sK + C.fdx * v) * C.inv2g;
  const float eEf = e + off, eWf = e - off;
  const float uEf = u + 0.5f * su, uWf = u - 0.5f * su;
  const float vEf = v + 0.5f * sv, vWf = v - 0.5f * sv;
  // face j+1/2: left = east face of this cell, right = west face of cell j+1
  float F0, F1, F2;
  cu_flux(eEf, uEf, vEf, lane_next(eWf), lane_next(uWf), lane_next(vWf), C, F0, F1, F2);
  d0 = F0 - lane_prev(F0);
  d1 = F1 - lane_prev(F1);  // x normal momentum = hu
  d2 = F2 - lane_prev(F2);  // x tangential momentum = hv
}

// y reconstruction of row k from rows k-1, k, k+1: north and south face states
// (eta, v = normal, u = tangential).
struct YFace {
  float e, n, t;
};
__device__ __forceinline__ void y_recon(float em, float um, float vm, float e, float u, float v,
                                        float ep, float up, float vp, const SweConst& C,
                                        YFace& N, YFace& S) {
  const float Lc = C.g * e;
  const float Lp = C.g * ep + C.hfdy * (u + up);
  const float Lm = C.g * em - C.hfdy * (u + um);
  const float sL = limited(Lm, Lc, Lp, C.theta);
  const float su = limited(um, u, up, C.theta);
  const float sv = limited(vm, v, vp, C.theta);
  const float off = (sL - C.fdy * u) * C.inv2g;
  N.e = e + off;
  S.e = e - off;
  N.n = v + 0.5f * sv;
  S.n = v - 0.5f * sv;
  N.t = u + 0.5f * su;
  S.t = u - 0.5f * su;
}

// One RK stage as a row pipeline: push row m (eta, hu, hv), emit row m-2 of
// psi + dt L(psi) (the forward-Euler part of the stage).
struct StagePipe {
  // rows m-2 ("a") and m-1 ("b")
  float ea, qa, ra, ua, va, ea_x0, ea_x1, ea_x2;
  float eb, qb, rb, ub, vb, eb_x0, eb_x1, eb_x2;
  YFace Na;          // north face state of row m-2
  float g0, g1, g2;  // y flux at face (m-2) - 1/2: mass, hv (normal), hu (tangential)

  __device__ __forceinline__ void push(float e, float q, float r, const SweConst& C, float& oe,
                                       float& oq, float& orr) {
    const float rh = rcpf(C.H + e);
    const float u = q * rh, v = r * rh;
    float x0, x1, x2;
    x_divergence(e, u, v, C, x0, x1, x2);
    YFace Nb, Sb;
    y_recon(ea, ua, va, eb, ub, vb, e, u, v, C, Nb, Sb);  // row m-1
    float G0, G1, G2;                                     // face (m-2) + 1/2
    cu_flux(Na.e, Na.n, Na.t, Sb.e, Sb.n, Sb.t, C, G0, G1, G2);
    const float dt = C.dt;
    oe = ea + dt * (-ea_x0 * C.idx - (G0 - g0) * C.idy);
    oq = qa + dt * (-ea_x1 * C.idx - (G2 - g2) * C.idy + C.f * ra);
    orr = ra + dt * (-ea_x2 * C.idx - (G1 - g1) * C.idy - C.f * qa);
    // advance
    ea = eb; qa = qb; ra = rb; ua = ub; va = vb;
    ea_x0 = eb_x0; ea_x1 = eb_x1; ea_x2 = eb_x2;
    eb = e; qb = q; rb = r; ub = u; vb = v;
    eb_x0 = x0; eb_x1 = x1; eb_x2 = x2;
    Na = Nb;
    g0 = G0; g1 = G1; g2 = G2;
  }
};

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__global__ __launch_bounds__(256) void swe_substep_kernel(const float* __restrict__ in,
                                                          float* __restrict__ out, SweConst C,
                                                          int total_waves) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wave >= total_waves) return;  // whole wave exits together
  const int per_particle = C.n_strip_x * C.n_strip_y;
  const int particle = wave / per_particle;
  const int rem = wave - particle * per_particle;
  const int sy = rem / C.n_strip_x;
  const int sx = rem - sy * C.n_strip_x;
  const int nx = C.nx, ny = C.ny;
  const size_t ncell = (size_t)nx * ny;
  const float* Ein = in + (size_t)particle * 3 * ncell;
  const float* Qin = Ein + ncell;
  const float* Rin = Qin + ncell;
  float* Eout = out + (size_t)particle * 3 * ncell;
  float* Qout = Eout + ncell;
  float* Rout = Qout + ncell;

  const int j = sx * kSweOut + lane - kSweHalo;  // unwrapped column
  const int jw = wrap(j, nx);
  const bool writer = lane >= kSweHalo && lane < kWave - kSweHalo && j < nx;
  const int k0 = sy * C.strip_h;
  const int k_end = min(k0 + C.strip_h, ny);  // exclusive
  const int m_first = k0 - 4, m_last = k_end + 3;

  StagePipe s1 = {}, s2 = {};
  // psi^n ring for the stage-2 combination: rows m-4 .. m-1 after a push of row m
  float pe4 = 0, pq4 = 0, pr4 = 0, pe3 = 0, pq3 = 0, pr3 = 0, pe2 = 0, pq2 = 0, pr2 = 0;
  float pe1 = 0, pq1 = 0, pr1 = 0;

  size_t off = (size_t)wrap(m_first, ny) * nx + jw;
  float ne_ = Ein[off], nq_ = Qin[off], nr_ = Rin[off];
  for (int m = m_first; m <= m_last; ++m) {
    const float e = ne_, q = nq_, r = nr_;
    if (m < m_last) {  // prefetch the next row
      const size_t o2 = (size_t)wrap(m + 1, ny) * nx + jw;
      ne_ = Ein[o2];
      nq_ = Qin[o2];
      nr_ = Rin[o2];
    }
    float se, sq, sr;
    s1.push(e, q, r, C, se, sq, sr);  // psi* of row m - 2 (valid for m >= k0)
    // psi^n ring: before the shift p*4 holds row m-4, the row stage 2 emits below
    const float qe4 = pe4, qq4 = pq4, qr4 = pr4;
    pe4 = pe3; pq4 = pq3; pr4 = pr3;
    pe3 = pe2; pq3 = pq2; pr3 = pr2;
    pe2 = pe1; pq2 = pq1; pr2 = pr1;
    pe1 = e; pq1 = q; pr1 = r;
    if (m >= k0) {
      float te, tq, tr;
      s2.push(se, sq, sr, C, te, tq, tr);  // psi* + dt L(psi*) of row m - 4
      if (m >= k0 + 4 && writer) {
        const size_t o = (size_t)(m - 4) * nx + j;
        Eout[o] = 0.5f * (qe4 + te);
        Qout[o] = 0.5f * (qq4 + tq);
        Rout[o] = 0.5f * (qr4 + tr);
      }
    }
  }
}

}  // namespace

void launch_swe_substep(const SweConst& C, int ne, const float* in, float* out, hipStream_t s) {
  const int total = ne * C.n_strip_x * C.n_strip_y;
  const int blocks = (total + 3) / 4;
  hipLaunchKernelGGL(swe_substep_kernel, dim3(blocks), dim3(256), 0, s, in, out, C, total);
}

}  // namespace iewpf
