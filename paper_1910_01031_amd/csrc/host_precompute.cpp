// Host-side float64 precompute done once per context (iewpf_create):
//   * SOAR stencils (eq. soar_function, eq. local_soar_on_eta) and q0 from a pointwise std;
//   * pull windows: the response Q^{1/2} Q^{1/2,T} H^T e_b of one observation to the unit
//     vectors e_1 = (1, 0), e_2 = (0, 1) (eq. detailedOPDUpdate read right to left):
//     adjoint geostrophic dipole on a coarse grid centred on the observed cell (eq.
//     adjointGeoBalance, coefficient g H / f), SOAR twice, Catmull-Rom interpolation to the
//     fine cells, central-difference geostrophic balance (eq. geostrophic_balance_disc).
//     Because the coarse grid is re-centred on every observation, the response depends
//     only on the offset from the observed cell; it is computed once on the infinite plane
//     and folded onto the torus when the grid is smaller than the window;
//   * H Q H^T read off the windows at the centre and S = (H Q H^T + R)^{-1} via Cholesky
//     (eq. S_extended);
//   * the local 7x7-block operator A = I - Q_S G^T H^T S_c H G Q_S on the coarse grid used
//     as model grid (fig. localsvd) and its symmetric square root by cyclic Jacobi.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace iewpf {

void soar_stencil(double q0, double L0, double dxc, double dyc, double out[25]) {
  for (int q = -2; q <= 2; ++q)
    for (int p = -2; p <= 2; ++p) {
      const double d = std::sqrt((p * dxc) * (p * dxc) + (q * dyc) * (q * dyc));
      out[(q + 2) * 5 + (p + 2)] = q0 * (1.0 + d / L0) * std::exp(-d / L0);
    }
}

double soar_q0(double std_, double L0, double dxc, double dyc) {
  double k[25];
  soar_stencil(1.0, L0, dxc, dyc, k);
  double s = 0.0;
  for (double v : k) s += v * v;
  return std_ / std::sqrt(s);
}

int inverse_spd2(const double A[4], double out[4]) {
  // Cholesky A = L L^T of the symmetrised 2x2, then A^{-1} = L^{-T} L^{-1}.
  const double a = A[0], b = 0.5 * (A[1] + A[2]), d = A[3];
  if (!(a > 0.0)) return -1;
  const double l11 = std::sqrt(a);
  const double l21 = b / l11;
  const double t = d - l21 * l21;
  if (!(t > 0.0)) return -1;
  const double l22 = std::sqrt(t);
  // L^{-1} = [[1/l11, 0], [-l21/(l11 l22), 1/l22]]
  const double i11 = 1.0 / l11, i22 = 1.0 / l22, i21 = -l21 / (l11 * l22);
  out[0] = i11 * i11 + i21 * i21;
  out[1] = i21 * i22;
  out[2] = i21 * i22;
  out[3] = i22 * i22;
  return 0;
}

namespace {

// Catmull-Rom (cubic convolution, a = -1/2) weights for taps -1, 0, 1, 2 at phase t.
void cr_weights(double t, double w[4]) {
  const double t2 = t * t, t3 = t2 * t;
  w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
  w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
  w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
  w[3] = 0.5 * (t3 - t2);
}

int floor_div(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// Plane coarse field: adjoint geostrophic dipole of s = (su, sv) (coarse spacing).
// Returns values on offsets [-R, R]^2, R given, index (n + R) * (2R+1) + (m + R).
void coarse_dipole(double su, double sv, double a, double dxc, double dyc, int R,
                   std::vector<double>& out) {
  const int W = 2 * R + 1;
  out.assign(W * W, 0.0);
  auto at = [&](int m, int n) -> double& { return out[(n + R) * W + (m + R)]; };
  at(0, 1) += -a * su / (2.0 * dyc);
  at(0, -1) += a * su / (2.0 * dyc);
  at(1, 0) += a * sv / (2.0 * dxc);
  at(-1, 0) += -a * sv / (2.0 * dxc);
}

// Plane SOAR convolution of a field on [-R, R]^2 producing [-(R+2), R+2]^2.
void soar_plane(const std::vector<double>& in, int R, const double w[25], std::vector<double>& out) {
  const int Ro = R + 2, Wi = 2 * R + 1, Wo = 2 * Ro + 1;
  out.assign(Wo * Wo, 0.0);
  for (int n = -Ro; n <= Ro; ++n)
    for (int m = -Ro; m <= Ro; ++m) {
      double acc = 0.0;
      for (int q = -2; q <= 2; ++q)
        for (int p = -2; p <= 2; ++p) {
          const int mm = m + p, nn = n + q;
          if (mm < -R || mm > R || nn < -R || nn > R) continue;
          acc += w[(q + 2) * 5 + (p + 2)] * in[(nn + R) * Wi + (mm + R)];
        }
      out[(n + Ro) * Wo + (m + Ro)] = acc;
    }
}

// Symmetric eigen-decomposition by cyclic Jacobi rotations (row-major n x n).
void jacobi_eigen(int n, std::vector<double> a, std::vector<double>& lam, std::vector<double>& v) {
  v.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? diag : off) += a[i * n + j] * a[i * n + j];
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[p * n + p], aqq = a[q * n + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = a[i * n + i];
}

}  // namespace

int build_pull_windows(const iewpf_ctx& ctx, double* out, double M[4]) {
  const iewpf_config& cf = ctx.cfg;
  const int c = ctx.c;
  const double dxc = c * cf.dx, dyc = c * cf.dy;
  const double a = cf.g * cf.H / cf.f;
  const int r = 7 * c;              // window radius in fine cells
  const int W = 2 * r + 1;
  const int Re = 7 * c - 1;         // eta extent before the geostrophic difference
  const int We = 2 * Re + 1;
  const int RZ = 5;                 // coarse extent: dipole 1 + SOAR 2 + SOAR 2
  for (int b = 0; b < 2; ++b) {
    std::vector<double> D, Z1, Z2;
    coarse_dipole(b == 0 ? 1.0 : 0.0, b == 0 ? 0.0 : 1.0, a, dxc, dyc, 1, D);
    soar_plane(D, 1, ctx.soar_me, Z1);
    soar_plane(Z1, 3, ctx.soar_me, Z2);  // Z2 on [-5, 5]^2
    const int WZ = 2 * RZ + 1;
    auto zat = [&](int m, int n) -> double {
      if (m < -RZ || m > RZ || n < -RZ || n > RZ) return 0.0;
      return Z2[(n + RZ) * WZ + (m + RZ)];
    };
    // eta on fine offsets [-Re, Re]^2 by Catmull-Rom from the observation-centred grid
    std::vector<double> eta(We * We, 0.0);
    for (int dy = -Re; dy <= Re; ++dy) {
      const int by = floor_div(dy, c);
      double wyv[4];
      cr_weights(static_cast<double>(dy - by * c) / c, wyv);
      for (int dx = -Re; dx <= Re; ++dx) {
        const int bx = floor_div(dx, c);
        double wxv[4];
        cr_weights(static_cast<double>(dx - bx * c) / c, wxv);
        double acc = 0.0;
        for (int n = 0; n < 4; ++n) {
          double row = 0.0;
          for (int m = 0; m < 4; ++m) row += wxv[m] * zat(bx + m - 1, by + n - 1);
          acc += wyv[n] * row;
        }
        eta[(dy + Re) * We + (dx + Re)] = acc;
      }
    }
    auto eat = [&](int dx, int dy) -> double {
      if (dx < -Re || dx > Re || dy < -Re || dy > Re) return 0.0;
      return eta[(dy + Re) * We + (dx + Re)];
    };
    // full window on the plane, then fold onto the stored extents
    for (int f = 0; f < 3; ++f) {
      double* dst = out + (size_t)(b * 3 + f) * ctx.wy * ctx.wx;
      for (int i = 0; i < ctx.wy * ctx.wx; ++i) dst[i] = 0.0;
    }
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const double e = eat(dx, dy);
        const double hu = -a * (eat(dx, dy + 1) - eat(dx, dy - 1)) / (2.0 * cf.dy);
        const double hv = a * (eat(dx + 1, dy) - eat(dx - 1, dy)) / (2.0 * cf.dx);
        const int ix = ctx.rx >= 0 ? dx + ctx.rx : ((dx % ctx.nx) + ctx.nx) % ctx.nx;
        const int iy = ctx.ry >= 0 ? dy + ctx.ry : ((dy % ctx.ny) + ctx.ny) % ctx.ny;
        const double vals[3] = {e, hu, hv};
        for (int f = 0; f < 3; ++f) out[((size_t)(b * 3 + f) * ctx.wy + iy) * ctx.wx + ix] += vals[f];
      }
  }
  (void)W;
  // H Q H^T: (hu, hv) of the two responses at the observed cell (offset 0, 0)
  const int cx = ctx.rx >= 0 ? ctx.rx : 0, cy = ctx.ry >= 0 ? ctx.ry : 0;
  for (int b = 0; b < 2; ++b)
    for (int f = 0; f < 2; ++f)
      M[f * 2 + b] = out[((size_t)(b * 3 + 1 + f) * ctx.wy + cy) * ctx.wx + cx];
  return 0;
}

int build_local_block(const iewpf_ctx& ctx, double ahalf[49 * 49], double Sc[4]) {
  const iewpf_config& cf = ctx.cfg;
  const double dxc = ctx.c * cf.dx, dyc = ctx.c * cf.dy;
  const double a = cf.g * cf.H / cf.f;
  // K rows: (H G_c Q_S)^T e_b = Q_S (adjoint coarse dipole of e_b), on [-3, 3]^2
  std::vector<double> K[2];
  for (int b = 0; b < 2; ++b) {
    std::vector<double> D;
    coarse_dipole(b == 0 ? 1.0 : 0.0, b == 0 ? 0.0 : 1.0, a, dxc, dyc, 1, D);
    soar_plane(D, 1, ctx.soar_me, K[b]);
  }
  double Mc[4];
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      double s = 0.0;
      for (int i = 0; i < 49; ++i) s += K[p][i] * K[q][i];
      Mc[p * 2 + q] = s;
    }
  double MR[4] = {Mc[0] + cf.obs_sigma * cf.obs_sigma, Mc[1], Mc[2],
                  Mc[3] + cf.obs_sigma * cf.obs_sigma};
  if (inverse_spd2(MR, Sc) != 0) return -1;
  std::vector<double> A(49 * 49);
  for (int i = 0; i < 49; ++i)
    for (int j = 0; j < 49; ++j) {
      double bij = 0.0;
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) bij += K[p][i] * Sc[p * 2 + q] * K[q][j];
      A[i * 49 + j] = (i == j ? 1.0 : 0.0) - bij;
    }
  std::vector<double> lam, V;
  jacobi_eigen(49, A, lam, V);
  for (int i = 0; i < 49; ++i)
    for (int j = 0; j < 49; ++j) {
      double s = 0.0;
      for (int k = 0; k < 49; ++k) s += V[i * 49 + k] * std::sqrt(std::fmax(lam[k], 0.0)) * V[j * 49 + k];
      ahalf[i * 49 + j] = s;
    }
  return 0;
}

void fill_cr_table(int c, CrTable& t) {
  for (int p = 0; p < 2 * kCrMaxC; ++p) {
    double w[4] = {0.0, 0.0, 0.0, 0.0};
    if (c <= kCrMaxC && p < 2 * c) cr_weights(static_cast<double>(p) / (2.0 * c), w);
    for (int m = 0; m < 4; ++m) t.w[p][m] = static_cast<float>(w[m]);
  }
}

}  // namespace iewpf
