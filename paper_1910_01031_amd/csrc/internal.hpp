// Internal declarations of the IEWPF HIP library: context layout, kernel constants and
// launchers.  Everything here is private to libiewpf.so; the public ABI is iewpf.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "iewpf.h"
#include "swe_const.hpp"

#include <vector>

namespace iewpf {

// ---- error reporting -------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define IEWPF_HIP_TRY(expr)                                                             \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::iewpf::fail(IEWPF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---- constants passed by value to kernels ----------------------------------------------

// Coarse random grid and covariance stencils.
struct CoarseConst {
  int nx, ny;          // fine grid
  int c;               // coarsening
  int nrx, nry;        // coarse grid
  float gb_x, gb_y;    // g H / (2 f dx), g H / (2 f dy)
};

// Observation / pull-window geometry for the analysis update.
struct PullConst {
  int wx, wy;          // stored window extents
  int ws;              // window row stride per field in floats (device layout [wy][6][ws])
  int rx, ry;          // window radii (-1: folded onto the whole period)
  int simple_x;        // rx >= 0 and nx >= wx + kWave: update entries carry lane 0's offset
  int n_obs;
  int strip_h, n_strip_x, n_strip_y;
};

// Device window row stride per field for windows up to this wide (a compile-time stride lets
// the six field loads of one window cell take immediate offsets).
constexpr int kWinStride = 128;
inline int window_stride(int wx) { return wx <= kWinStride ? kWinStride : wx; }

// Analysis status words: int32 [4] at byte offset 8 * kScalStatus of the analysis scalars
// (scal): [0] flags set by the sync kernel, [1] the first particle with a non-finite scalar
// (or -1), [2] flags set by the update pass, [3] the first particle with a non-finite
// updated value (0x7fffffff if none).  The posterior and update kernels write nothing when
// [0] has kStatSkipUpdate bits, so such an analysis leaves the state untouched.
constexpr int kScalStatus = 8;
constexpr int kStatBeta = 1;             // two-stage beta <= 0 (eq. betaTwoStage)
constexpr int kStatNonfiniteScalar = 2;  // c_i, gamma_i, zeta_i, c*_i or alpha_i not finite
constexpr int kStatSkipUpdate = kStatBeta | kStatNonfiniteScalar;
constexpr int kStatNonfiniteState = 4;   // a value written by the update is not finite

constexpr int kGbHalo = 1;                    // lanes lost per side by the geostrophic stencil
constexpr int kGbOut = kWave - 2 * kGbHalo;    // 62 output columns per wave
constexpr int kBlockN = 49;                   // 7x7 local block of the posterior operator

}  // namespace iewpf

// ---- the context ------------------------------------------------------------------------
struct iewpf_ctx {
  iewpf_config cfg;
  int nx, ny, c, nrx, nry, nr, ne, max_obs;
  size_t ncell;            // nx * ny
  double n_psi;            // 3 nx ny
  // host-side precompute (float64)
  double q0_me, q0_init;
  double soar_me[25], soar_init[25];
  double S[4], Sc[4], Mfine[4];
  double ahalf[iewpf::kBlockN * iewpf::kBlockN];
  int wx, wy, rx, ry;      // pull window geometry
  int ws = 128;            // device window row stride per field (window_stride(wx))
  bool simple_x = false;   // see PullConst::simple_x
  iewpf::SweConst swe;       // the scheme step's form for this context's launches
  iewpf::SweConst swe_halo;  // the strip form (batched launches use it)
  iewpf::CoarseConst cc;
  float soar_me_f[25], soar_init_f[25];
  // device workspaces
  float* scratch = nullptr;    // one state-sized buffer [ne][3][ny][nx]
  float* xi = nullptr;         // [ne][nr]
  float* nu = nullptr;         // [ne][nr]
  float* coarse = nullptr;     // [ne][nr] SOAR output / r'
  float* coarse2 = nullptr;    // [ne][nr]
  // model-error fields of up to me_chunk consecutive model steps, drawn by one normals and
  // one SOAR launch: [me_chunk][ne][nr] each
  float* me_xi = nullptr;
  float* me_coarse = nullptr;
  int me_chunk = 1;
  float* windows = nullptr;    // [wy][6][window_stride(wx)]: (s_u, s_v) x (eta, hu, hv)
  float* wcell = nullptr;      // the same, cell-major [wy][wx][6], when they fit in LDS
  float* dmat = nullptr;       // A^{1/2} - I, float32 [49][49]
  double* sd = nullptr;        // [ne][max_obs][2]
  double* vblk = nullptr;      // posterior block products [ne][max_obs][49]
  double* pcoef = nullptr;     // posterior coefficients per particle [ne][3]
  float* sdf = nullptr;        // S d rounded to float32, [max_obs + 1][sd_float_stride(ne)][2]
                               // (row max_obs stays zero: the update lists' sentinel)
  double* cval = nullptr;      // [ne]
  double* dots = nullptr;      // [ne][3]
  double* part_dots = nullptr; // [ne][parts][3] partial dot products
  double* alpha = nullptr;     // [ne]
  double* cstar = nullptr;     // [ne]
  double* scal = nullptr;      // [16] analysis scalars
  int32_t* obs_cells = nullptr;  // [max_obs][2]
  double* obs_y = nullptr;       // [max_obs][2]
  int32_t* pt_off = nullptr;     // coarse-point CSR offsets [nr + 1]
  int32_t* pt_ent = nullptr;     // entries (obs << 8 | block index) [max_obs * 49]
  // update lists per column strip: entries (window column, window row, obs, 0), each
  // column's observations sorted by window row and listed twice [n_upd_cols * 2 * max_obs][4];
  // st_off [n_upd_cols + 1] their CSR offsets; st_rows [n_upd_cols][ny][2] per row the
  // entry range whose windows hold the row
  int32_t* st_off = nullptr;
  int32_t* st_rows = nullptr;
  int32_t* st_ent = nullptr;
  int n_upd_cols = 0;
  int upd_strip_h = 16;
  int gb_strip_h = 6;
  bool use_lds = false;          // the update stages its windows in LDS (wcell)
  double* dk1 = nullptr;         // drifter k1 [ne][max_obs][2]
  double* dpstar = nullptr;      // drifter p*  [ne][max_obs][2]
  double* dobs = nullptr;        // observation synthesis output [max_obs][2]
  unsigned* cflmax = nullptr;    // 2 words
  int32_t* dparents = nullptr;  // resampling scratch [ne]
  int32_t* sir_parents = nullptr;  // parents of the last SIR analysis [ne]
  int32_t* dobs_cells = nullptr;   // drifter observation synthesis: cells [max_obs][2]
  double* dcum = nullptr;       // resampling: cumulative residuals [ne]
  // pinned host staging
  unsigned char* h_stage = nullptr;
  size_t stage_bytes = 0;
  // device copy of the staging area, same layout: obs_cells, obs_y, pt_off, pt_ent, st_off
  // and st_ent point into it, so one analysis uploads its observation lists in one copy
  unsigned char* d_stage = nullptr;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  double* h_small = nullptr;     // small pinned readback buffer
  // pinned, device-mapped: the sync kernel writes the analysis scalars and status words here
  // (kScalStatus doubles, then 5 int32: the status words and the update's error flag) when
  // publish_host is set, so a synchronous analysis needs no copy back
  double* h_sync = nullptr;
  bool publish_host = false;
  // device address of the pinned staging area (it is mapped); y_use: where the analysis reads
  // the observation values when not from the device staging block (a synchronous analysis with
  // unchanged cells reads them straight from the pinned staging area, no upload)
  unsigned char* h_stage_dev = nullptr;
  const double* y_use = nullptr;
  int last_n_obs = 0;
  // optional per-launch event trace
  bool trace = false;
  int n_trace = 0;
  hipEvent_t* trace_ev = nullptr;   // [2 * kTraceMax]
  int* trace_kind = nullptr;        // [kTraceMax]
  // surrogate window: saved input states and per-particle drift / flags
  float* saved = nullptr;
  double* sdrift = nullptr;
  int32_t* sflags = nullptr;
  float* wstart = nullptr;  // surrogate drifter forecast: the state at the window start
  // full innovation covariance (optional): float64 windows, S [2 n]^2 of the cached cell set,
  // work matrix, raw innovations, status word
  bool full_innov = false;
  int one_stage = 0;  // 1: the one-stage scheme (target max c, no nu term)
  int sir = 0;        // 1: the standard particle filter (SIR weights, residual resampling)
  double* windows64 = nullptr;
  double* fS = nullptr;
  double* fX = nullptr;
  double* dinn = nullptr;
  int32_t* fstatus = nullptr;
  std::vector<int32_t> f_cells;  // cells the cached S was built for
  int f_n = -1;
  // cells whose observation lists (and cells) are on the device in d_stage; -1: none
  std::vector<int32_t> list_cells;
  int list_n = -1;
  std::vector<double> h_win64;  // float64 pull windows [2][3][wy][wx] (host copy)
};

namespace iewpf {
constexpr int kTraceMax = 8192;
enum TraceKind {
  kTrSubstep = 0, kTrNormals, kTrSoar, kTrGbAdd, kTrInnov, kTrRandDots, kTrSync,
  kTrPosterior, kTrUpdate, kTrSubstepNoise, kTrSoarMe, kTrKinds
};
// Records a start event (returns the slot or -1) and the matching stop event.
int trace_begin(iewpf_ctx* c, int kind, hipStream_t s);
void trace_end(iewpf_ctx* c, int slot, hipStream_t s);
struct TraceScope {
  iewpf_ctx* c;
  int slot;
  hipStream_t s;
  TraceScope(iewpf_ctx* c_, int kind, hipStream_t s_) : c(c_), slot(trace_begin(c_, kind, s_)), s(s_) {}
  ~TraceScope() { trace_end(c, slot, s); }
};
}  // namespace iewpf

// ---- host precompute (host_precompute.cpp) ----------------------------------------------
namespace iewpf {
double soar_q0(double std_, double L0, double dxc, double dyc);
void soar_stencil(double q0, double L0, double dxc, double dyc, double out[25]);
// Pull windows for s = e_1 and s = e_2; out[6][wy][wx], plus the 2x2 H Q H^T at the centre.
int build_pull_windows(const iewpf_ctx& ctx, double* out, double M[4]);
// Local posterior block: A^{1/2} [49x49] and S_c.
int build_local_block(const iewpf_ctx& ctx, double ahalf[49 * 49], double Sc[4]);
int inverse_spd2(const double A[4], double out[4]);
}  // namespace iewpf

// ---- surrogate network (surrogate_kernels.hip, surrogate_api.cpp) ----------------------------
namespace iewpf {
enum ConvIn { kInStateNorm = 0, kInNhwcVec = 1, kInNhwcSmall = 2 };
enum ConvOut { kOutReluBf16 = 0, kOutResidState = 1, kOutF32 = 2, kOutMaskBf16 = 3 };
struct ConvArgs {
  int B, H, W;             // images and grid
  int cin, cout;           // channels
  int K, Kpad, Npad;       // K = 9 cin, padded to 32; output channels padded to 16
  const void* in;          // kInStateNorm: float [B][3][H][W]; else bf16 [B][H][W][cin]
  const uint16_t* wt;      // bf16 [Npad][Kpad]
  const float* bias;       // [cout] or nullptr
  void* out;               // by output mode
  const float* state_in;   // kOutResidState: psi, float [B][3][H][W]
  const uint16_t* mask;    // kOutMaskBf16: activation whose sign masks the output
  float mu[3], isig[3], s[3];
};
void launch_conv(const ConvArgs& A, int in_mode, int out_mode, hipStream_t s);
// Two consecutive layers in one pass (A: -> 48 channels with ReLU, B: 48 -> ...); false when
// the shapes have no fused kernel (the caller then runs them one by one).
bool launch_conv_pair(const ConvArgs& LA, int in_mode, const ConvArgs& LB, int out_mode,
                      hipStream_t s);
int net_max_cells(const iewpf_net* n);
int net_horizon(const iewpf_net* n);
void launch_wgrad(const ConvArgs& A, int in_mode, const uint16_t* g, int gch, int cells_per_chunk,
                  float* part, hipStream_t s);
void launch_bgrad(const uint16_t* g, int gch, int ncells, int cells_per_chunk, float* part,
                  hipStream_t s);
void launch_reduce_grads(const float* wpart, const float* bpart, int nchunks, int cin, int cout,
                         int Kpad, int Npad, float* gw, float* gb, hipStream_t s);
void launch_mse(const float* y, const float* st_in, const float* st_tgt, int B, int H, int W,
                const float sc[3], uint16_t* g, float* lpart, int nblocks, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t s);
void launch_prep_weights(const float* w, int cin, int cout, int Kf, int Npf, int Kd, int Npd,
                         uint16_t* wf, uint16_t* wd, hipStream_t s);
void launch_mass_drift(const float* before, const float* after, int ne, int ncell, double H,
                       double tol, double* drift, int32_t* flags, hipStream_t s);
// out[0] = number of nonzero flags[0 .. n)
void launch_count_flags(const int32_t* flags, int n, int32_t* out, hipStream_t s);
// dst particle i = src particle i for every i with flags[i] != 0 (per floats per particle)
void launch_copy_flagged(const float* src, float* dst, const int32_t* flags, int ne, size_t per,
                         hipStream_t s);
// per-channel normalisation statistics of training pairs: out = {mu[3], sigma[3], scale[3]}
// (float64, device); part holds channel_stats_parts() doubles
int channel_stats_parts();
void launch_channel_stats(const float* x, const float* t, int B, int hw, double* part, double* out,
                          hipStream_t s);
}  // namespace iewpf

// ---- launchers (kernels in *.hip) ---------------------------------------------------------
namespace iewpf {
// resident waves per compute unit of the stencil / analysis-update kernels (occupancy)
int swe_waves_per_cu();
// workgroups of the full-row form (nx columns) resident per compute unit
int swe_row_blocks_per_cu(int nx);
int update_waves_per_cu();
int update_particle_group();
// Number of row strips for a wave-per-strip kernel: minimises (launch rounds) x (rows a
// wave marches), rounds = ceil(columns * n_strips / slots), rows = ceil(ny / n_strips) +
// halo_rows.  columns = strips per row of strips (all particles).
int choose_row_strips(int columns, int ny, int slots, int halo_rows, int min_rows);
// noise: each job adds the model-error field zstep of its chunk (job.z + zstep job.z_field)
void launch_swe_batch(const SweJobTable* tab, int total_waves, int parity, bool noise, int zstep,
                      hipStream_t s);
// z != nullptr: also add the model error Q_GB I_Omega z (z: [ne][nry][nrx] SOAR field);
// mask != nullptr (plain steps only, z == nullptr): only particles i with mask[i] != 0 are
// stepped (the others' workgroups return at once and their output is not written)
void launch_swe_substep(const SweConst& C, int ne, const float* in, float* out, const float* z,
                        hipStream_t s, const int32_t* mask = nullptr);
// n_steps fields [n_steps][ne][n], field t drawn for step index step + t
void launch_normals(float* out, int n, int ne, uint64_t seed, uint64_t step, uint32_t tag,
                    uint32_t ens, hipStream_t s, const uint64_t* dyn = nullptr, int n_steps = 1);
void launch_soar(const CoarseConst& C, const float* w25, int ne, const float* in, float* out,
                 hipStream_t s);
// psi (+)= Q_GB I_Omega z  [+ pull];  base != nullptr: psi = base + ...
void launch_gb_add(const CoarseConst& C, int ne, const float* z, const float* base, float* psi,
                   int strip_h, hipStream_t s);
// Particles per wave of the analysis update; sdf pads the particle count to a multiple of it.
#ifndef IEWPF_UPD_PB
#define IEWPF_UPD_PB 4
#endif
constexpr int kUpdParticles = IEWPF_UPD_PB;
inline int sd_float_stride(int ne) {
  return (ne + kUpdParticles - 1) / kUpdParticles * kUpdParticles;
}
// wcell (cell-major windows [wy * wx][6], or null): stage the windows in LDS
void launch_analysis_update(const CoarseConst& C, const PullConst& P, int ne, const float* z,
                            const float* windows, const float* wcell, const float* sdf,
                            const int32_t* st_rows, const int32_t* st_ent, float* psi,
                            double* scal, int32_t* host_flag, hipStream_t s);
// LDS of the staged-window update (two workgroups fit one compute unit up to this size)
constexpr size_t kUpdateLdsMax = 80 * 1024;
size_t update_lds_bytes(int wx, int wy);
// cell-major windows plus one zero cell in float4s, padded to whole 64-float4 chunks (the
// device copy has this length)
__host__ __device__ inline int update_lds_float4s(int wx, int wy) {
  return ((6 * (wx * wy + 1) + 3) / 4 + 63) / 64 * 64;
}
int update_lds_waves_per_cu();
// c_i = out_scale * sum_o d^T S d (out_scale = -1/2 and S = R^{-1} give the log-weights of
// the standard particle filter); sdf (may be null) receives S d in float32, observation-major
void launch_innovation(int ne, int n_obs, int max_obs, int nx, int ny, double H, const double S[4],
                       const float* psi, const int32_t* cells, const double* y, double* sd,
                       float* sdf, double* cval, hipStream_t s, double out_scale = 1.0);
void launch_sir_normalise(int ne, const double* logw, double* w, hipStream_t s);
void launch_observe_drifters(int n, int nx, int ny, double dx, double dy, double H, double sigma,
                             double dt_obs, uint64_t seed, uint64_t step, uint32_t ens,
                             const double* pos_now, const double* pos_prev, int32_t* cells,
                             double* y, hipStream_t s);
int rand_dots_parts();
// innovations, S d, c_i and the draws with their per-part dot products in one launch
void launch_innov_draws(int ne, int n_obs, int max_obs, int nx, int ny, double H,
                        const double S[4], const float* psi, const int32_t* cells, const double* y,
                        double* sd, float* sdf, double* cval, int nr, uint64_t seed, uint64_t step,
                        uint32_t ens, float* xi, float* nu, double* part_dots, hipStream_t s,
                        const uint64_t* dyn = nullptr);
// xi, nu~ and their per-part dot products (summed by the sync kernel)
void launch_rand_dots(int ne, int nr, uint64_t seed, uint64_t step, uint32_t ens, float* xi,
                      float* nu, double* part_dots, hipStream_t s, const uint64_t* dyn = nullptr);
// Full innovation covariance: assemble sym(H Q H^T) + sigma^2 I [2 n_obs]^2 (float64) from the
// float64 pull windows, factor it A = L L^T in place in one workgroup (n <= chol_max_order();
// lower triangle L, upper L^T), solve A x = b per right-hand side (rhs == nullptr gives the
// columns of S = A^{-1}; with rhs, x = S b and cval = b^T S b), and S d, c_i = d^T S d for
// every particle from the explicit S.
void launch_hqht_full(int n_obs, int nx, int ny, int rx, int ry, int wx, int wy, const double* win,
                      const int32_t* cells, double sigma2, double* M, hipStream_t s);
int chol_max_order();
void launch_chol_factor(int n, double* A, int32_t* status, hipStream_t s);
void launch_chol_solve(int n, int nrhs, const double* L, const double* rhs, int rhs_stride,
                       double* out, int out_stride, double* cval, hipStream_t s);
void launch_sd_full(int n, int ne, int stride, const double* S, const double* D, double* SD,
                    float* sdf, double* cval, hipStream_t s);
// Also writes the analysis status words (kScalStatus) that the posterior and update kernels
// check before writing.
void launch_sync(int ne, int nr, double n_psi, int one_stage, const double* cval,
                 const double* part_dots, double* dots, double* alpha, double* cstar,
                 double* scal, double* host_out, hipStream_t s);
// vblk: [ne][max_obs][49] block products (A^{1/2} - I) r of every observation's block;
// coef: [ne][3] the coefficients of r per particle
void launch_posterior_coarse(const CoarseConst& C, int ne, int n_obs, int max_obs,
                             const int32_t* cells, const float* xi, const float* nu,
                             const double* dots, const double* alpha, const double* scal,
                             const float* dmat, const int32_t* pt_off, const int32_t* pt_ent,
                             double* vblk, double* coef, float* rout, hipStream_t s);
void launch_observe(int n_obs, int nx, int ny, double H, double sigma, uint64_t seed,
                    uint64_t step, uint32_t ens, const float* truth, const int32_t* cells,
                    double* y, hipStream_t s);
void launch_cfl(int ne, int nx, int ny, float H, float g, const float* psi, unsigned* out,
                hipStream_t s);
// psi_b, w: the velocity is taken from psi + w (psi_b - psi) (psi_b NULL: from psi)
void launch_drift_k1(int ne, int nd, int nx, int ny, double dx, double dy, double H, double dt,
                     const float* psi, const double* pos, double* k1, double* pstar,
                     hipStream_t s, const float* psi_b = nullptr, double w = 0.0);
void launch_drift_k2(int ne, int nd, int nx, int ny, double dx, double dy, double H, double dt,
                     const float* psi, double* pos, const double* k1, const double* pstar,
                     double* traj, hipStream_t s, const float* psi_b = nullptr, double w = 0.0);
void launch_resample(int ne, uint64_t seed, uint64_t step, uint32_t ens, const double* logw,
                     int32_t* parents, int32_t* counts, double* cum, hipStream_t s,
                     double* scal = nullptr);
void launch_gather_particles(int ne, size_t per_particle, const int32_t* parents, const float* in,
                             float* out, hipStream_t s);

// Batched cycles: the per-cycle inputs (observation values of every ensemble, the step and
// analysis counters) copied by one kernel from pinned, device-mapped host memory into the
// contexts' device buffers, and the ensembles' analysis status words gathered by one kernel
// into pinned host memory; so a captured cycle holds no copy nodes.
struct BatchStageIn {
  const double* y_src[kMaxBatch];  // device-mapped pinned values, 2 n_obs per ensemble
  double* y_dst[kMaxBatch];        // the contexts' device observation values
  int n_y[kMaxBatch];              // doubles per ensemble
  const uint64_t* dyn_src;         // 2 counters (device-mapped) or nullptr
  uint64_t* dyn_dst;
};
void launch_batch_stage_in(const BatchStageIn& a, int n, hipStream_t s);
struct BatchStatusOut {
  const int32_t* src[kMaxBatch];  // each ensemble's 4 status words
  int32_t* dst;                   // device-mapped pinned [n][4]
};
void launch_batch_status(const BatchStatusOut& a, int n, hipStream_t s);
}  // namespace iewpf
