// Constants and tables of the shallow-water scheme kernels (passed by value or read from a
// device table).  Kept apart from the other internals: everything the scheme kernels'
// code depends on is in swe_kernels.hip, this header and buffer_dev.hpp.
#pragma once

#include <cstddef>

namespace iewpf {

constexpr int kWave = 64;
constexpr int kSweHalo = 4;                   // lanes lost per side by the fused RK stages
constexpr int kSweOut = kWave - 2 * kSweHalo;  // 56 output columns per wave

// Catmull-Rom weights of the interpolation I_Omega (taps -1, 0, 1, 2) at the phases
// t = p / (2c), p = 0 .. 2c-1, of fine rows between coarse points (filled on the host in
// float64, rounded once).  Contexts accept c <= kCrMaxC.
constexpr int kCrMaxC = 16;
struct CrTable {
  float w[2 * kCrMaxC][4];
};
void fill_cr_table(int c, CrTable& t);

// Shallow-water scheme constants (float32, as used by the stencil).
struct SweConst {
  int nx, ny;
  int row;             // 1: full-row form (one workgroup per row strip, nx <= 512)
  int strip_h;         // rows per wave strip
  int n_strip_x, n_strip_y;
  float H, g, inv2g, f;
  float hfdx, hfdy;    // f dx / 2, f dy / 2 (Coriolis potential increments)
  float fdx, fdy;      // f dx, f dy
  float theta;
  // the limiter works on slopes divided by theta; these fold theta back in
  float k2t;           // 1 / (2 theta): the central difference's weight in the minmod
  float ht;            // theta / 2: face offset of u, v per limited slope
  float fxg, fyg;      // f dx / (2 g), f dy / (2 g): Coriolis potential / g increments
  float dt, idx, idy;  // scheme step, 1/dx, 1/dy
  float dtidx, dtidy, dtf;  // dt/dx, dt/dy, dt f
  // fused model error (last scheme step of a model step)
  int c, nrx, nry;     // coarsening and coarse grid
  float gb_x, gb_y;    // g H / (2 f dx), g H / (2 f dy)
  CrTable cr;          // interpolation weights by phase
};

// One ensemble of a batched stencil launch (device-resident table).
struct SweJob {
  SweConst C;
  const float* z;   // fused model-error fields (first of a chunk of model steps) or nullptr
  size_t z_field;   // floats per model step's field (n_particles nry nrx)
  float* buf_a;     // the caller's state
  float* buf_b;     // the context's scratch state
  int wave_begin;
};
constexpr int kMaxBatch = 16;
struct SweJobTable {
  int n;
  int total_waves;
  SweJob job[kMaxBatch];
};

}  // namespace iewpf
