// extern "C" entry points of libiewpf.so (declared in include/iewpf.h).
//
// The host side validates arguments, keeps the float64 precompute, builds the per-call
// observation index lists (which observation windows touch which fine strip, which 7x7
// blocks touch which coarse point) and enqueues kernels; every arithmetic step of the
// forecast and the analysis runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

struct iewpf_batch {
  int n = 0;
  std::vector<iewpf_ctx*> ctx;
  std::vector<float*> state;
  std::vector<int> n_obs;
  std::vector<size_t> y_off;     // offsets into the pinned y buffer
  iewpf::SweJobTable* tab_plain = nullptr;  // device tables
  iewpf::SweJobTable* tab_noise = nullptr;
  int total_waves = 0;
  bool split = false;             // one launch per ensemble (each in its own form) per scheme step
  int n_sub = 1;
  uint64_t* d_dyn = nullptr;      // device counters: first step, analysis index
  uint64_t* h_dyn = nullptr;      // pinned
  double* h_y = nullptr;          // pinned observation values
  int32_t* h_status = nullptr;    // pinned analysis status words, 4 per ensemble
  // device addresses of the three pinned buffers (they are mapped): the cycle's first kernel
  // reads the values and counters there, its last one writes the status words there
  const double* h_y_dev = nullptr;
  const uint64_t* h_dyn_dev = nullptr;
  int32_t* h_status_dev = nullptr;
  size_t h_y_len = 0;
  hipEvent_t copy_ev = nullptr;
  bool copy_pending = false;
  hipStream_t gs = nullptr;       // capture / replay stream
  hipEvent_t in_ev = nullptr, out_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_steps = -1;
  // side streams (default priority) for the per-ensemble work that does not depend on the
  // other ensembles (model-error fields, analyses): forked from and joined back into the
  // cycle's stream, so in a captured graph they become parallel branches
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> fork_ev;  // one per fork point
  std::vector<hipEvent_t> join_ev;  // one per side stream and fork point
};

namespace iewpf {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int trace_begin(iewpf_ctx* c, int kind, hipStream_t s) {
  if (!c->trace || c->n_trace >= kTraceMax) return -1;
  const int slot = c->n_trace++;
  c->trace_kind[slot] = kind;
  (void)hipEventRecord(c->trace_ev[2 * slot], s);
  return slot;
}

void trace_end(iewpf_ctx* c, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(c->trace_ev[2 * slot + 1], s);
}

int choose_row_strips(int columns, int ny, int slots, int halo_rows, int min_rows) {
  int best = 1;
  double best_cost = 1e300;
  const int max_strips = std::max(1, ny / std::max(1, min_rows));
  for (int n = 1; n <= max_strips; ++n) {
    const long long waves = (long long)columns * n;
    const long long rounds = (waves + slots - 1) / slots;
    const int rows = (ny + n - 1) / n + halo_rows;
    const double cost = (double)rounds * rows;
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = n;
    }
  }
  return best;
}

namespace {

constexpr uint32_t kTagModelError = 1;
constexpr uint32_t kTagInit = 5;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <class T>
int dev_alloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
  if (e != hipSuccess) return fail(IEWPF_E_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  return 0;
}

int env_int(const char* name, int def) {
  const char* v = std::getenv(name);
  if (!v || !*v) return def;
  return std::atoi(v);
}

void free_ctx(iewpf_ctx* c) {
  if (!c) return;
  void* bufs[] = {c->windows64, c->fS, c->fX, c->dinn, c->fstatus, c->me_xi, c->me_coarse,
                  c->wstart, c->saved, c->sdrift, c->sflags, c->scratch, c->part_dots, c->xi, c->nu,
                  c->coarse, c->coarse2, c->windows,
                  c->dmat,    c->sd,     c->cval,   c->dots,   c->alpha,   c->cstar,
                  c->scal,    c->d_stage, c->dk1,    c->dpstar, c->dobs,   c->cflmax,  c->dparents,
                  c->dcum,    c->sir_parents, c->dobs_cells, c->sdf, c->wcell, c->vblk, c->pcoef};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->h_small) (void)hipHostFree(c->h_small);
  if (c->h_sync) (void)hipHostFree(c->h_sync);
  if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
  if (c->trace_ev) {
    for (int i = 0; i < 2 * kTraceMax; ++i)
      if (c->trace_ev[i]) (void)hipEventDestroy(c->trace_ev[i]);
    delete[] c->trace_ev;
  }
  delete[] c->trace_kind;
  delete c;
}

// Circular distance from point p to the half-open interval [a, a + len) on Z_n.
int circ_interval_dist(int p, int a, int len, int n) {
  int d = (p - a) % n;
  if (d < 0) d += n;
  if (d < len) return 0;
  return std::min(d - (len - 1), n - d);
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

struct StageLayout {
  size_t cells, y, pt_off, pt_ent, st_off, st_rows, st_ent, total;
};

StageLayout stage_layout(const iewpf_ctx& c) {
  StageLayout L;
  size_t o = 0;
  L.cells = o; o = align16(o + sizeof(int32_t) * 2 * c.max_obs);
  L.y = o; o = align16(o + sizeof(double) * 2 * c.max_obs);
  L.pt_off = o; o = align16(o + sizeof(int32_t) * (c.nr + 1));
  L.pt_ent = o; o = align16(o + sizeof(int32_t) * (size_t)c.max_obs * kBlockN);
  L.st_off = o; o = align16(o + sizeof(int32_t) * (c.n_upd_cols + 1));
  L.st_rows = o; o = align16(o + sizeof(int32_t) * 2 * (size_t)c.n_upd_cols * c.ny);
  L.st_ent = o; o = align16(o + sizeof(int32_t) * 4 * (1 + 2 * (size_t)c.n_upd_cols * c.max_obs));
  L.total = o;
  return L;
}

int device_slots(int waves_per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return cus * waves_per_cu;
}

int wait_stage(iewpf_ctx* c) {
  if (c->stage_pending) {
    IEWPF_HIP_TRY(hipEventSynchronize(c->stage_ev));
    c->stage_pending = false;
  }
  return 0;
}

int check_cells(const iewpf_ctx* c, const int32_t* cells, int n) {
  for (int o = 0; o < n; ++o) {
    if (cells[2 * o] < 0 || cells[2 * o] >= c->nx || cells[2 * o + 1] < 0 ||
        cells[2 * o + 1] >= c->ny)
      return fail(IEWPF_E_ARG, "observation cell out of the grid");
  }
  return 0;
}

// psi += Q^{1/2} xi for every particle, xi from stream (step, model-error tag).
void add_noise(iewpf_ctx* c, float* psi, uint64_t step, hipStream_t s) {
  {
    TraceScope t(c, kTrNormals, s);
    launch_normals(c->xi, c->nr, c->ne, c->cfg.seed, step, kTagModelError, c->cfg.ensemble_id, s);
  }
  {
    TraceScope t(c, kTrSoar, s);
    launch_soar(c->cc, c->soar_me_f, c->ne, c->xi, c->coarse, s);
  }
  TraceScope t(c, kTrGbAdd, s);
  launch_gb_add(c->cc, c->ne, c->coarse, nullptr, psi, c->gb_strip_h, s);
}

// One model-error draw (stream `step`, tag 1) with the SOAR weights scaled by `scale`.
void add_scaled_noise(iewpf_ctx* c, float* psi, uint64_t step, double scale, hipStream_t s) {
  float w[25];
  for (int q = 0; q < 25; ++q) w[q] = (float)(scale * c->soar_me[q]);
  launch_normals(c->xi, c->nr, c->ne, c->cfg.seed, step, kTagModelError, c->cfg.ensemble_id, s);
  launch_soar(c->cc, w, c->ne, c->xi, c->coarse, s);
  launch_gb_add(c->cc, c->ne, c->coarse, nullptr, psi, c->gb_strip_h, s);
}

// Builds the per-call observation index lists from the cells in the pinned staging area
// and uploads cells (and y when with_y) and the lists on the stream.
//   coarse point -> (observation, 7x7 block row) pairs, ascending observations per point
//   update column strip and row -> observations whose pull window holds the row
int upload_observations(iewpf_ctx* c, int n_obs, bool with_y, hipStream_t s,
                        bool y_mapped = false) {
  const StageLayout L = stage_layout(*c);
  int32_t* cells = reinterpret_cast<int32_t*>(c->h_stage + L.cells);
  if (with_y && n_obs == c->list_n &&
      std::equal(cells, cells + 2 * n_obs, c->list_cells.begin())) {
    // same cells as the lists on the device (moorings): only the values go up, or (y_mapped,
    // a caller that waits for the analysis before it returns) the kernels read them from the
    // pinned staging area
    if (y_mapped && c->h_stage_dev) {
      c->y_use = reinterpret_cast<const double*>(c->h_stage_dev + L.y);
      c->last_n_obs = n_obs;
      return 0;
    }
    if (n_obs > 0)
      IEWPF_HIP_TRY(hipMemcpyAsync(c->d_stage + L.y, c->h_stage + L.y, sizeof(double) * 2 * n_obs,
                                   hipMemcpyHostToDevice, s));
    IEWPF_HIP_TRY(hipEventRecord(c->stage_ev, s));
    c->stage_pending = true;
    c->last_n_obs = n_obs;
    return 0;
  }
  int32_t* pt_off = reinterpret_cast<int32_t*>(c->h_stage + L.pt_off);
  int32_t* pt_ent = reinterpret_cast<int32_t*>(c->h_stage + L.pt_ent);
  std::fill(pt_off, pt_off + c->nr + 1, 0);
  auto block_point = [&](int o, int q) {
    const int ao = cells[2 * o] / c->c, bo = cells[2 * o + 1] / c->c;
    const int pa = ((ao + q % 7 - 3) % c->nrx + c->nrx) % c->nrx;
    const int pb = ((bo + q / 7 - 3) % c->nry + c->nry) % c->nry;
    return pb * c->nrx + pa;
  };
  for (int o = 0; o < n_obs; ++o)
    for (int q = 0; q < kBlockN; ++q) pt_off[block_point(o, q) + 1]++;
  for (int p = 0; p < c->nr; ++p) pt_off[p + 1] += pt_off[p];
  {
    std::vector<int32_t> fillp(pt_off, pt_off + c->nr);
    for (int o = 0; o < n_obs; ++o)
      for (int q = 0; q < kBlockN; ++q) pt_ent[fillp[block_point(o, q)]++] = (o << 8) | q;
  }
  // Update lists, per column strip of the update kernel: the observations whose pull window
  // reaches the strip's columns, sorted by the window's first row and listed twice (the
  // second time one period further down), so that the windows holding a row k are the
  // consecutive entries whose (unwrapped) first row lies in (k + ny - wy, k + ny]; st_rows
  // holds that range for every row.  Entry 0 is a sentinel (zero S d row, no window column)
  // that pads the kernel's last batch of a row.  An entry holds the window's column (with
  // simple_x the byte offset of lane 0's cell in the strided window row, lane 0 sitting at
  // column j0 - kGbHalo; else the window's first column), its first row, the byte offset of
  // the observation's S d row, and with simple_x lane 0's byte offset in a cell-major row.
  const int nsx = (c->nx + kGbOut - 1) / kGbOut;
  const int ne4 = sd_float_stride(c->ne);
  int32_t* st_off = reinterpret_cast<int32_t*>(c->h_stage + L.st_off);
  int32_t* st_rows = reinterpret_cast<int32_t*>(c->h_stage + L.st_rows);
  int32_t* st_ent = reinterpret_cast<int32_t*>(c->h_stage + L.st_ent);
  st_ent[0] = c->simple_x ? 4 * c->wx : 0;
  st_ent[1] = 0;
  st_ent[2] = (int32_t)(sizeof(float) * 2 * (size_t)ne4 * c->max_obs);
  st_ent[3] = 24 * c->wx;
  int t = 1;
  st_off[0] = t;
  std::vector<std::pair<int, int>> col;  // (window row, observation)
  for (int sx = 0; sx < nsx; ++sx) {
    const int j0 = sx * kGbOut;
    const int lenj = std::min(kGbOut, c->nx - j0);
    col.clear();
    for (int o = 0; o < n_obs; ++o) {
      if (c->rx >= 0 && circ_interval_dist(cells[2 * o], j0, lenj, c->nx) > c->rx) continue;
      // the window's first row on the torus (a window folded onto the whole period starts at
      // the observed cell)
      const int ko = cells[2 * o + 1];
      col.emplace_back(c->ry < 0 ? ko : ((ko - c->ry) % c->ny + c->ny) % c->ny, o);
    }
    std::stable_sort(col.begin(), col.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                       return a.first < b.first;
                     });
    const int n = (int)col.size(), base = t;
    for (int rep = 0; rep < 2; ++rep)
      for (const auto& q : col) {
        const int jo = cells[2 * q.second];
        const int js = c->rx < 0 ? jo : ((jo - c->rx) % c->nx + c->nx) % c->nx;
        int32_t* e = st_ent + 4 * (size_t)t++;
        e[0] = js;
        e[3] = 0;
        if (c->simple_x) {
          // lane l's window column is (l + a) mod nx; no lane wraps when a + 63 < nx, and
          // otherwise the lanes that do not wrap lie past the window (a > nx - 64 >= wx):
          // lane 0's column offset a' in bytes of the strided window rows (4 a') and of
          // the cell-major LDS rows (24 a')
          const int a = ((j0 - kGbHalo - js) % c->nx + c->nx) % c->nx;
          const int a1 = a + kWave - 1 < c->nx ? a : a - c->nx;
          e[0] = 4 * a1;
          e[3] = 24 * a1;
        }
        e[1] = q.first;
        e[2] = (int32_t)(sizeof(float) * 2 * (size_t)ne4 * q.second);
      }
    st_off[sx + 1] = t;
    // unwrapped first row of doubled entry i
    auto row_of = [&](int i) { return i < n ? col[i].first : col[i - n].first + c->ny; };
    int lo = 0, hi = 0;
    for (int k = 0; k < c->ny; ++k) {
      const int kk = k + c->ny;
      while (lo < 2 * n && row_of(lo) <= kk - c->wy) ++lo;
      while (hi < 2 * n && row_of(hi) <= kk) ++hi;
      st_rows[2 * ((size_t)sx * c->ny + k)] = base + lo;
      st_rows[2 * ((size_t)sx * c->ny + k) + 1] = base + std::max(lo, hi);
    }
  }
  // One copy of the staging area up to the last used list entry (the device block has the
  // same layout): small transfers each cost a fixed latency on the stream, so one copy of
  // the whole prefix beats six copies of the used parts.  Without y, the y block is skipped
  // (the caller uploads y itself) with a second copy from pt_off on.
  const size_t end = L.st_ent + sizeof(int32_t) * 4 * (size_t)t;
  if (with_y) {
    IEWPF_HIP_TRY(hipMemcpyAsync(c->d_stage, c->h_stage, end, hipMemcpyHostToDevice, s));
  } else {
    IEWPF_HIP_TRY(hipMemcpyAsync(c->d_stage + L.cells, c->h_stage + L.cells, L.y - L.cells,
                                 hipMemcpyHostToDevice, s));
    IEWPF_HIP_TRY(hipMemcpyAsync(c->d_stage + L.pt_off, c->h_stage + L.pt_off, end - L.pt_off,
                                 hipMemcpyHostToDevice, s));
  }
  IEWPF_HIP_TRY(hipEventRecord(c->stage_ev, s));
  c->stage_pending = true;
  c->last_n_obs = n_obs;
  c->list_cells.assign(cells, cells + 2 * n_obs);
  c->list_n = n_obs;
  return 0;
}

// Full innovation covariance for the observed cells (already on the device): rebuilt and
// factored only when the cell set differs from the cached one; waits for the stream then.
int prepare_full_s(iewpf_ctx* c, const int32_t* cells, int n_obs, hipStream_t s) {
  if (n_obs == c->f_n && std::equal(cells, cells + 2 * n_obs, c->f_cells.begin())) return 0;
  const double s2 = c->cfg.obs_sigma * c->cfg.obs_sigma;
  launch_hqht_full(n_obs, c->nx, c->ny, c->rx, c->ry, c->wx, c->wy, c->windows64, c->obs_cells, s2,
                   c->fS, s);
  launch_chol_factor(2 * n_obs, c->fS, c->fstatus, s);
  // S = A^{-1} explicitly (columns from unit right-hand sides), kept with the factor
  launch_chol_solve(2 * n_obs, 2 * n_obs, c->fS, nullptr, 0, c->fX, 2 * n_obs, nullptr, s);
  IEWPF_HIP_TRY(hipGetLastError());
  int32_t st = 0;
  IEWPF_HIP_TRY(hipMemcpyAsync(&st, c->fstatus, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  if (st != 0) {
    c->f_n = -1;
    return fail(IEWPF_E_ARG, "full H Q H^T + R is not positive definite");
  }
  c->f_cells.assign(cells, cells + 2 * n_obs);
  c->f_n = n_obs;
  return 0;
}

// Return code of an analysis from its status words (host copy): non-finite scalars first
// (nothing was written), then beta <= 0 (nothing was written), then non-finite values written
// by the update.  `who` prefixes the message (the ensemble of a batch).
int analysis_status(const int32_t* st, const std::string& who) {
  if (st[0] & kStatNonfiniteScalar)
    return fail(IEWPF_E_NONFINITE, who + "non-finite c_i, gamma_i, zeta_i, c*_i or alpha_i in particle " +
                                       std::to_string(st[1]) + "; the state was not updated");
  if (st[0] & kStatBeta)
    return fail(IEWPF_E_BETA, who + "beta <= 0: ensemble violates N_psi >> N_y; the state was not updated");
  if (st[2] & kStatNonfiniteState)
    return fail(IEWPF_E_NONFINITE, who + "non-finite value in the analysed state of particle " +
                                       std::to_string(st[3]));
  return 0;
}

// The analysis kernels of one ensemble on the observations already on the device.
// dyn: device counters (dyn[1] = analysis index added to analysis_index) or nullptr.
int launch_analysis(iewpf_ctx* c, float* state, int n_obs, uint64_t analysis_index,
                    const uint64_t* dyn, hipStream_t s) {
  if (c->sir) {
    // standard particle filter: l_i = -1/2 sum_o d^T R^{-1} d, residual resampling, and the
    // parents' states gathered through the scratch buffer
    const double r = c->cfg.obs_sigma * c->cfg.obs_sigma;
    const double Rinv[4] = {1.0 / r, 0.0, 0.0, 1.0 / r};
    launch_innovation(c->ne, n_obs, c->max_obs, c->nx, c->ny, c->cfg.H, Rinv, state, c->obs_cells,
                      c->y_use ? c->y_use : c->obs_y, c->sd, nullptr, c->cval, s, -0.5);
    launch_resample(c->ne, c->cfg.seed, analysis_index, c->cfg.ensemble_id, c->cval, c->sir_parents,
                    c->dparents, c->dcum, s, c->scal);
    const size_t per = 3 * c->ncell;
    launch_gather_particles(c->ne, per, c->sir_parents, state, c->scratch, s);
    IEWPF_HIP_TRY(hipMemcpyAsync(state, c->scratch, sizeof(float) * per * c->ne,
                                 hipMemcpyDeviceToDevice, s));
    IEWPF_HIP_TRY(hipGetLastError());
    return 0;
  }
  if (c->full_innov && n_obs > 0) {
    // stages 1-2: raw d, then S d and c_i with the full S
    {
      TraceScope tr(c, kTrInnov, s);
      const double I2[4] = {1.0, 0.0, 0.0, 1.0};
      launch_innovation(c->ne, n_obs, c->max_obs, c->nx, c->ny, c->cfg.H, I2, state, c->obs_cells,
                        c->y_use ? c->y_use : c->obs_y, c->dinn, nullptr, c->cval, s);
      launch_sd_full(2 * n_obs, c->ne, 2 * c->max_obs, c->fX, c->dinn, c->sd, c->sdf, c->cval, s);
    }
    // stage 3: xi, nu~ and their dot products
    TraceScope tr(c, kTrRandDots, s);
    launch_rand_dots(c->ne, c->nr, c->cfg.seed, analysis_index, c->cfg.ensemble_id, c->xi, c->nu,
                     c->part_dots, s, dyn);
  } else {
    // stages 1-3 in one launch: innovations, S d, c_i and the draws with their dot products
    TraceScope tr(c, kTrRandDots, s);
    launch_innov_draws(c->ne, n_obs, c->max_obs, c->nx, c->ny, c->cfg.H, c->S, state,
                       c->obs_cells, c->y_use ? c->y_use : c->obs_y, c->sd, c->sdf, c->cval,
                       c->nr, c->cfg.seed,
                       analysis_index,
                       c->cfg.ensemble_id, c->xi, c->nu, c->part_dots, s, dyn);
  }
  // stages 4-5: cbar, beta, c*, alpha (the one ensemble-wide step)
  {
    TraceScope tr(c, kTrSync, s);
    launch_sync(c->ne, c->nr, c->n_psi, c->one_stage, c->cval, c->part_dots, c->dots, c->alpha,
                c->cstar, c->scal, c->publish_host ? c->h_sync : nullptr, s);
  }
  // stage 6: r' on the coarse grid, SOAR, then one fused pass over the state
  {
    TraceScope tr(c, kTrPosterior, s);
    launch_posterior_coarse(c->cc, c->ne, n_obs, c->max_obs, c->obs_cells, c->xi, c->nu, c->dots,
                            c->alpha, c->scal, c->dmat, c->pt_off, c->pt_ent, c->vblk,
                            c->pcoef, c->coarse2, s);
  }
  {
    TraceScope tr(c, kTrSoar, s);
    launch_soar(c->cc, c->soar_me_f, c->ne, c->coarse2, c->coarse, s);
  }
  PullConst P;
  P.wx = c->wx;
  P.wy = c->wy;
  P.ws = c->ws;
  P.simple_x = c->simple_x ? 1 : 0;
  P.rx = c->rx;
  P.ry = c->ry;
  P.n_obs = n_obs;
  P.strip_h = c->upd_strip_h;
  P.n_strip_x = (c->nx + kGbOut - 1) / kGbOut;
  P.n_strip_y = (c->ny + c->upd_strip_h - 1) / c->upd_strip_h;
  {
    TraceScope tr(c, kTrUpdate, s);
    launch_analysis_update(
        c->cc, P, c->ne, c->coarse, c->windows, c->wcell, c->sdf, c->st_rows, c->st_ent, state,
        c->scal,
        c->publish_host ? reinterpret_cast<int32_t*>(c->h_sync + kScalStatus) + 4 : nullptr, s);
  }
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int model_steps(iewpf_ctx* c, float* state, int n_steps, uint64_t first_step, int noise_on_last,
                hipStream_t s) {
  float* cur = state;
  float* other = c->scratch;
  const size_t field = (size_t)c->ne * c->nr;
  const int n_noise = noise_on_last ? n_steps : n_steps - 1;  // model error after steps 0 .. n_noise-1
  int chunk0 = 0, chunk_n = 0;  // the fields of steps chunk0 .. chunk0 + chunk_n - 1 are drawn
  for (int st = 0; st < n_steps; ++st) {
    const bool noise = st < n_noise;
    if (noise && st >= chunk0 + chunk_n) {
      // coarse fields z = SOAR xi of the next model steps, each added by the last scheme
      // step of its model step; one launch of each kernel for the whole chunk
      chunk0 = st;
      chunk_n = std::min(c->me_chunk, n_noise - st);
      {
        TraceScope t(c, kTrNormals, s);
        launch_normals(c->me_xi, c->nr, c->ne, c->cfg.seed, first_step + st, kTagModelError,
                       c->cfg.ensemble_id, s, nullptr, chunk_n);
      }
      TraceScope t(c, kTrSoarMe, s);
      launch_soar(c->cc, c->soar_me_f, c->ne * chunk_n, c->me_xi, c->me_coarse, s);
    }
    const float* z = noise ? c->me_coarse + (size_t)(st - chunk0) * field : nullptr;
    for (int sub = 0; sub < c->cfg.n_sub; ++sub) {
      const bool fuse = noise && sub == c->cfg.n_sub - 1;
      {
        TraceScope t(c, fuse ? kTrSubstepNoise : kTrSubstep, s);
        launch_swe_substep(c->swe, c->ne, cur, other, fuse ? z : nullptr, s);
      }
      std::swap(cur, other);
    }
  }
  if (cur != state)
    IEWPF_HIP_TRY(hipMemcpyAsync(state, cur, sizeof(float) * 3 * c->ncell * c->ne,
                                 hipMemcpyDeviceToDevice, s));
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

// Runs body(e, stream) for every ensemble e, spread over the batch's side streams after
// everything already on s, and makes s wait for all of them.  `point` numbers the fork so
// that every fork of one cycle has its own events.
template <class F>
int batch_fork(iewpf_batch* b, int point, hipStream_t s, F&& body) {
  const int k = (int)b->side.size();
  while ((int)b->fork_ev.size() <= point) {
    hipEvent_t ev;
    IEWPF_HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->fork_ev.push_back(ev);
    for (int i = 0; i < k; ++i) {
      IEWPF_HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      b->join_ev.push_back(ev);
    }
  }
  IEWPF_HIP_TRY(hipEventRecord(b->fork_ev[point], s));
  for (int i = 0; i < k; ++i) IEWPF_HIP_TRY(hipStreamWaitEvent(b->side[i], b->fork_ev[point], 0));
  for (int e = 0; e < b->n; ++e)
    if (int rc = body(e, b->side[e % k])) return rc;
  for (int i = 0; i < k; ++i) {
    hipEvent_t j = b->join_ev[(size_t)point * k + i];
    IEWPF_HIP_TRY(hipEventRecord(j, b->side[i]));
    IEWPF_HIP_TRY(hipStreamWaitEvent(s, j, 0));
  }
  return 0;
}

// Model steps of every ensemble of a batch; dyn != nullptr reads the first step index
// from dyn[0] (the kernels then see step offsets only).
int batch_model_steps(iewpf_batch* b, int n_steps, uint64_t first_step, const uint64_t* dyn,
                      hipStream_t s) {
  int parity = 0;
  const int n_noise = n_steps - 1;  // model error after every step but the last
  int chunk_max = n_noise;
  for (int e = 0; e < b->n; ++e) chunk_max = std::min(chunk_max, b->ctx[e]->me_chunk);
  int chunk0 = 0, chunk_n = 0, fork = 0;
  for (int st = 0; st < n_steps; ++st) {
    const bool noise = st < n_noise;
    if (noise && st >= chunk0 + chunk_n) {
      // the model-error fields of the next model steps of every ensemble, drawn ahead by one
      // normals and one SOAR launch per ensemble (the same draws as one launch per step)
      chunk0 = st;
      chunk_n = std::min(chunk_max, n_noise - st);
      const int rc = batch_fork(b, fork++, s, [&](int e, hipStream_t es) {
        iewpf_ctx* c = b->ctx[e];
        launch_normals(c->me_xi, c->nr, c->ne, c->cfg.seed, (dyn ? 0 : first_step) + st,
                       kTagModelError, c->cfg.ensemble_id, es, dyn, chunk_n);
        launch_soar(c->cc, c->soar_me_f, c->ne * chunk_n, c->me_xi, c->me_coarse, es);
        return 0;
      });
      if (rc) return rc;
    }
    for (int sub = 0; sub < b->n_sub; ++sub) {
      const bool fuse = noise && sub == b->n_sub - 1;
      if (b->split) {
        // every ensemble's own launch, in its own form, as parallel branches
        const int rc = batch_fork(b, n_steps + 1 + st * b->n_sub + sub, s, [&](int e, hipStream_t es) {
          iewpf_ctx* c = b->ctx[e];
          float* in = parity ? c->scratch : b->state[e];
          float* out = parity ? b->state[e] : c->scratch;
          const float* z = fuse ? c->me_coarse + (size_t)(st - chunk0) * c->ne * c->nr : nullptr;
          launch_swe_substep(c->swe, c->ne, in, out, z, es);
          return 0;
        });
        if (rc) return rc;
      } else {
        launch_swe_batch(fuse ? b->tab_noise : b->tab_plain, b->total_waves, parity, fuse,
                         fuse ? st - chunk0 : 0, s);
      }
      parity ^= 1;
    }
  }
  if (parity)
    for (int e = 0; e < b->n; ++e)
      IEWPF_HIP_TRY(hipMemcpyAsync(b->state[e], b->ctx[e]->scratch,
                                   sizeof(float) * 3 * b->ctx[e]->ncell * b->ctx[e]->ne,
                                   hipMemcpyDeviceToDevice, s));
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int batch_cycle_body(iewpf_batch* b, int n_steps, uint64_t first_step, uint64_t analysis_index,
                     const uint64_t* dyn, hipStream_t s) {
  if (int rc = batch_model_steps(b, n_steps, first_step, dyn, s)) return rc;
  // fork points 0 .. n_steps - 1 are the model-error chunks (at most one per model step)
  return batch_fork(b, n_steps, s, [&](int e, hipStream_t es) {
    return launch_analysis(b->ctx[e], b->state[e], b->n_obs[e], dyn ? 0 : analysis_index, dyn, es);
  });
}

// A whole batched cycle on s: the observation values (and with dyn the counters) into the
// device buffers, the model steps and analyses, then every ensemble's status words into the
// pinned host buffer.  No copies: a captured cycle is kernels and stream joins only.
int batch_cycle_all(iewpf_batch* b, int n_steps, uint64_t first_step, uint64_t analysis_index,
                    bool dyn, hipStream_t s) {
  BatchStageIn in{};
  for (int e = 0; e < b->n; ++e) {
    in.y_src[e] = b->h_y_dev + b->y_off[e];
    in.y_dst[e] = b->ctx[e]->obs_y;
    in.n_y[e] = 2 * b->n_obs[e];
  }
  in.dyn_src = dyn ? b->h_dyn_dev : nullptr;
  in.dyn_dst = b->d_dyn;
  launch_batch_stage_in(in, b->n, s);
  if (int rc = batch_cycle_body(b, n_steps, first_step, analysis_index, dyn ? b->d_dyn : nullptr, s))
    return rc;
  BatchStatusOut out{};
  for (int e = 0; e < b->n; ++e)
    out.src[e] = reinterpret_cast<const int32_t*>(b->ctx[e]->scal + kScalStatus);
  out.dst = b->h_status_dev;
  launch_batch_status(out, b->n, s);
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

// Waits for a cycle on s and returns the first ensemble's error from the status words the
// cycle's last kernel wrote (an ensemble whose analysis failed before writing keeps its
// forecast state).
int batch_status(iewpf_batch* b, hipStream_t s) {
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  b->copy_pending = false;
  for (int e = 0; e < b->n; ++e)
    if (int rc = analysis_status(b->h_status + 4 * e, "ensemble " + std::to_string(e) + ": "))
      return rc;
  return 0;
}

void free_batch(iewpf_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->tab_plain) (void)hipFree(b->tab_plain);
  if (b->tab_noise) (void)hipFree(b->tab_noise);
  if (b->d_dyn) (void)hipFree(b->d_dyn);
  if (b->h_dyn) (void)hipHostFree(b->h_dyn);
  if (b->h_y) (void)hipHostFree(b->h_y);
  if (b->h_status) (void)hipHostFree(b->h_status);
  if (b->copy_ev) (void)hipEventDestroy(b->copy_ev);
  if (b->in_ev) (void)hipEventDestroy(b->in_ev);
  if (b->out_ev) (void)hipEventDestroy(b->out_ev);
  if (b->gs) (void)hipStreamDestroy(b->gs);
  for (hipStream_t x : b->side) (void)hipStreamDestroy(x);
  for (hipEvent_t x : b->fork_ev) (void)hipEventDestroy(x);
  for (hipEvent_t x : b->join_ev) (void)hipEventDestroy(x);
  delete b;
}

}  // namespace
}  // namespace iewpf

namespace iewpf {
namespace {
// The fastest strip height of one form of the scheme step on `state` (writes go to the
// context's scratch buffer).
int tune_strip(iewpf_ctx* c, const SweConst& form, const float* state, hipStream_t s,
               SweConst* best) {
  const int cands[] = {16, 24, 32, 40, 48, 60, 64, 75, 96};
  hipEvent_t e0, e1;
  IEWPF_HIP_TRY(hipEventCreate(&e0));
  IEWPF_HIP_TRY(hipEventCreate(&e1));
  *best = form;
  float best_ms = 1e30f;
  for (int h : cands) {
    if (h > c->ny && h != cands[0]) break;
    SweConst C = form;
    C.strip_h = std::min(h, c->ny);
    C.n_strip_y = (c->ny + C.strip_h - 1) / C.strip_h;
    launch_swe_substep(C, c->ne, state, c->scratch, nullptr, s);  // warm
    IEWPF_HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < 4; ++r) launch_swe_substep(C, c->ne, state, c->scratch, nullptr, s);
    IEWPF_HIP_TRY(hipEventRecord(e1, s));
    IEWPF_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    IEWPF_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      *best = C;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}
}  // namespace
}  // namespace iewpf

using namespace iewpf;

extern "C" {

const char* iewpf_last_error(void) { return g_last_error.c_str(); }

int iewpf_set_trace(iewpf_ctx* c, int on) {
  if (!c) return fail(IEWPF_E_ARG, "NULL argument");
  if (on && !c->trace_ev) {
    c->trace_ev = new hipEvent_t[2 * kTraceMax]();
    c->trace_kind = new int[kTraceMax]();
    for (int i = 0; i < 2 * kTraceMax; ++i)
      IEWPF_HIP_TRY(hipEventCreate(&c->trace_ev[i]));
  }
  c->trace = on != 0;
  c->n_trace = 0;
  return 0;
}

int iewpf_trace_read(iewpf_ctx* c, double* ms_out, int32_t* count_out, int n_kinds) {
  if (!c || !ms_out || !count_out || n_kinds < 0 || n_kinds > 16)
    return fail(IEWPF_E_ARG, "invalid argument");
  for (int k = 0; k < n_kinds; ++k) {
    ms_out[k] = 0.0;
    count_out[k] = 0;
  }
  for (int i = 0; i < c->n_trace; ++i) {
    IEWPF_HIP_TRY(hipEventSynchronize(c->trace_ev[2 * i + 1]));
    float ms = 0.0f;
    IEWPF_HIP_TRY(hipEventElapsedTime(&ms, c->trace_ev[2 * i], c->trace_ev[2 * i + 1]));
    const int k = c->trace_kind[i];
    if (k < n_kinds) {
      ms_out[k] += ms;
      count_out[k] += 1;
    }
  }
  return 0;
}

int iewpf_create(const iewpf_config* cfg, iewpf_ctx** out) {
  if (!cfg || !out) return fail(IEWPF_E_ARG, "NULL argument");
  *out = nullptr;
  const iewpf_config& f = *cfg;
  if (f.nx <= 0 || f.ny <= 0 || f.c_omega <= 0 || f.n_particles <= 0 || f.n_sub <= 0 ||
      !(f.dt > 0) || !(f.dx > 0) || !(f.dy > 0) || !(f.H > 0) || !(f.g > 0) || f.f == 0.0 ||
      !(f.obs_sigma > 0) || f.max_obs <= 0 || f.max_obs >= (1 << 22) || !(f.theta >= 1.0) ||
      !(f.theta <= 2.0) || f.me_std < 0 || f.init_std < 0 || f.n_particles > 65535)
    return fail(IEWPF_E_ARG, "invalid configuration value");
  if (f.c_omega > kCrMaxC)
    return fail(IEWPF_E_ARG, "c_omega above " + std::to_string(kCrMaxC) + " is not supported");
  if (f.nx % f.c_omega || f.ny % f.c_omega)
    return fail(IEWPF_E_SHAPE, "nx and ny must be divisible by c_omega");
  if (f.nx / f.c_omega < 7 || f.ny / f.c_omega < 7)
    return fail(IEWPF_E_SHAPE, "the coarse grid needs at least 7 points per direction");
  if (12.0 * f.nx * f.ny >= 2147483648.0)  // the scheme kernel addresses a particle's state in 31-bit bytes
    return fail(IEWPF_E_SHAPE, "nx ny above 178,956,970 cells per particle is not supported");
  // strip height of the scheme kernel (rows per wave); the environment may force it
  const int forced = env_int("IEWPF_SWE_STRIP", 32);
  if (forced < 1) return fail(IEWPF_E_ARG, "IEWPF_SWE_STRIP must be a positive number of rows");
  iewpf_ctx* c = new iewpf_ctx();
  c->cfg = f;
  c->nx = f.nx;
  c->ny = f.ny;
  c->c = f.c_omega;
  c->nrx = f.nx / f.c_omega;
  c->nry = f.ny / f.c_omega;
  c->nr = c->nrx * c->nry;
  c->ne = f.n_particles;
  c->max_obs = f.max_obs;
  c->ncell = (size_t)f.nx * f.ny;
  c->n_psi = 3.0 * (double)c->ncell;
  const double dxc = c->c * f.dx, dyc = c->c * f.dy;
  if (!(c->cfg.me_L0 > 0)) c->cfg.me_L0 = 0.75 * dxc;
  if (!(c->cfg.init_L0 > 0)) c->cfg.init_L0 = 0.75 * dxc;
  c->q0_me = soar_q0(f.me_std, c->cfg.me_L0, dxc, dyc);
  c->q0_init = soar_q0(f.init_std, c->cfg.init_L0, dxc, dyc);
  soar_stencil(c->q0_me, c->cfg.me_L0, dxc, dyc, c->soar_me);
  soar_stencil(c->q0_init, c->cfg.init_L0, dxc, dyc, c->soar_init);
  for (int i = 0; i < 25; ++i) {
    c->soar_me_f[i] = (float)c->soar_me[i];
    c->soar_init_f[i] = (float)c->soar_init[i];
  }
  // scheme constants
  SweConst& S = c->swe;
  S.nx = f.nx;
  S.ny = f.ny;
  S.n_strip_x = (f.nx + kSweOut - 1) / kSweOut;
  S.row = 0;
  {
    // rows per wave strip: fit the waves of all particles to the resident wave slots
    // (each wave marches strip_h + 8 rows of stage 1 and strip_h + 4 of stage 2)
    // 32 rows measured best on gfx950 at 500x300x100 (16..100 all within 10%); the
    // occupancy model only takes over when that would leave the GPU under-filled
    const int slots = device_slots(swe_waves_per_cu());
    int n_ys = (f.ny + forced - 1) / forced;
    if ((long long)S.n_strip_x * f.n_particles * n_ys < slots)
      n_ys = choose_row_strips(S.n_strip_x * f.n_particles, f.ny, slots, 6, 8);
    S.strip_h = (f.ny + n_ys - 1) / n_ys;
    S.n_strip_y = (f.ny + S.strip_h - 1) / S.strip_h;
  }
  S.H = (float)f.H;
  S.g = (float)f.g;
  S.inv2g = (float)(1.0 / (2.0 * f.g));
  S.f = (float)f.f;
  S.hfdx = (float)(0.5 * f.f * f.dx);
  S.hfdy = (float)(0.5 * f.f * f.dy);
  S.fdx = (float)(f.f * f.dx);
  S.fdy = (float)(f.f * f.dy);
  S.theta = (float)f.theta;
  S.k2t = (float)(1.0 / (2.0 * f.theta));
  S.ht = (float)(0.5 * f.theta);
  S.fxg = (float)(f.f * f.dx / (2.0 * f.g));
  S.fyg = (float)(f.f * f.dy / (2.0 * f.g));
  S.dt = (float)(f.dt / f.n_sub);
  S.idx = (float)(1.0 / f.dx);
  S.idy = (float)(1.0 / f.dy);
  S.dtidx = (float)(f.dt / f.n_sub / f.dx);
  S.dtidy = (float)(f.dt / f.n_sub / f.dy);
  S.dtf = (float)(f.dt / f.n_sub * f.f);
  S.c = c->c;
  S.nrx = c->nrx;
  S.nry = c->nry;
  S.gb_x = (float)(f.g * f.H / (2.0 * f.f * f.dx));
  S.gb_y = (float)(f.g * f.H / (2.0 * f.f * f.dy));
  c->swe_halo = S;
  {
    // Full-row form for rows of at most 512 columns when it computes sufficiently fewer
    // columns than the strip form (its three barriers per row cost ~10 % of issue rate):
    // lane use nx / (64 ceil(nx / 64)) against nx / (64 ceil(nx / 56)).
    const double use_row = (double)f.nx / (64.0 * ((f.nx + 63) / 64));
    const double use_halo = (double)f.nx / (64.0 * S.n_strip_x);
    const int choice = env_int("IEWPF_SWE_ROW", -1);
    const bool row = f.nx <= 512 && (choice == 1 || (choice < 0 && use_row >= 1.08 * use_halo));
    if (row) {
      // strips of rows: minimise (launch rounds) x (rows per workgroup + prologue rows)
      S.row = 1;
      const int forced_row = env_int("IEWPF_SWE_ROW_STRIP", 0);
      int n_ys;
      if (forced_row > 0) {
        n_ys = (f.ny + forced_row - 1) / forced_row;
      } else {
        int cus = 256, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
          cus = 256;
        n_ys = choose_row_strips(f.n_particles, f.ny, cus * swe_row_blocks_per_cu(f.nx), 8, 8);
      }
      S.strip_h = (f.ny + n_ys - 1) / n_ys;
      S.n_strip_y = (f.ny + S.strip_h - 1) / S.strip_h;
    }
  }
  c->cc.nx = f.nx;
  c->cc.ny = f.ny;
  c->cc.c = c->c;
  c->cc.nrx = c->nrx;
  c->cc.nry = c->nry;
  c->cc.gb_x = (float)(f.g * f.H / (2.0 * f.f * f.dx));
  c->cc.gb_y = (float)(f.g * f.H / (2.0 * f.f * f.dy));
  fill_cr_table(c->c, S.cr);
  c->swe_halo.cr = S.cr;
  // pull windows and S
  const int r = 7 * c->c, W = 2 * r + 1;
  c->rx = W > f.nx ? -1 : r;
  c->ry = W > f.ny ? -1 : r;
  c->wx = W > f.nx ? f.nx : W;
  c->wy = W > f.ny ? f.ny : W;
  c->ws = window_stride(c->wx);
  c->simple_x = c->rx >= 0 && f.nx >= c->wx + kWave;
  if (24.0 * c->ws * c->wy >= 2147483648.0) {  // the update kernel reads the windows in 31-bit bytes
    free_ctx(c);
    return fail(IEWPF_E_SHAPE, "pull windows above 2^31 bytes are not supported");
  }
  if (8.0 * sd_float_stride(f.n_particles) * (c->max_obs + 1.0) >= 2147483648.0) {
    free_ctx(c);  // the update lists address S d rows by 31-bit byte offsets
    return fail(IEWPF_E_CAPACITY, "particles x observations too large for the update lists");
  }
  std::vector<double> win((size_t)6 * c->wx * c->wy);
  build_pull_windows(*c, win.data(), c->Mfine);
  const double s2 = f.obs_sigma * f.obs_sigma;
  double MR[4] = {c->Mfine[0] + s2, c->Mfine[1], c->Mfine[2], c->Mfine[3] + s2};
  if (inverse_spd2(MR, c->S) != 0) {
    free_ctx(c);
    return fail(IEWPF_E_ARG, "H Q H^T + R is not positive definite");
  }
  if (build_local_block(*c, c->ahalf, c->Sc) != 0) {
    free_ctx(c);
    return fail(IEWPF_E_ARG, "coarse H Q H^T + R is not positive definite");
  }
  {
    // Update strips: every row's observation range comes with the lists, so a strip's
    // length costs only its two halo rows; the strips are sized for whole launch rounds
    // (IEWPF_UPD_STRIP forces a height).  Model-error strips: 6 rows.
    const int forced = env_int("IEWPF_UPD_STRIP", 0);
    const int groups = (c->ne + update_particle_group() - 1) / update_particle_group();
    const int nsx = (f.nx + kGbOut - 1) / kGbOut;
    c->use_lds = update_lds_bytes(c->wx, c->wy) <= kUpdateLdsMax && env_int("IEWPF_UPD_LDS", 1) != 0;
    const int slots =
        device_slots(c->use_lds ? update_lds_waves_per_cu() : update_waves_per_cu());
    int n_ys = forced > 0 ? (f.ny + forced - 1) / forced
                          : choose_row_strips(nsx * groups, f.ny, slots, 2, 4);
    // staged windows: strips of at most 8 rows (6-8 measured fastest for 100 particles on
    // 500x300, 12 % ahead of one launch round of 17-row strips)
    if (forced <= 0 && c->use_lds) n_ys = std::max(n_ys, (f.ny + 7) / 8);
    c->upd_strip_h = (f.ny + n_ys - 1) / n_ys;
    c->gb_strip_h = std::max(1, std::min(f.ny, env_int("IEWPF_GB_STRIP", 6)));
    c->n_upd_cols = nsx;
  }

  int rc = 0;
  const size_t nstate = 3 * c->ncell * (size_t)c->ne;
  rc |= dev_alloc(&c->scratch, nstate);
  rc |= dev_alloc(&c->xi, (size_t)c->ne * c->nr);
  rc |= dev_alloc(&c->nu, (size_t)c->ne * c->nr);
  rc |= dev_alloc(&c->coarse, (size_t)c->ne * c->nr);
  rc |= dev_alloc(&c->coarse2, (size_t)c->ne * c->nr);
  {
    // model-error fields drawn ahead: up to 16 model steps in about 64 MB, and at most 65535
    // fields per launch (the grid's y and z extents)
    const double field_bytes = 4.0 * c->ne * c->nr;
    const int cap = std::max(1, std::min(16, env_int("IEWPF_ME_CHUNK", 16)));
    c->me_chunk = (int)std::max(1.0, std::min((double)cap, std::floor(64.0 * (1 << 20) / field_bytes)));
    c->me_chunk = std::max(1, std::min(c->me_chunk, 65535 / c->ne));
  }
  rc |= dev_alloc(&c->me_xi, (size_t)c->me_chunk * c->ne * c->nr);
  rc |= dev_alloc(&c->me_coarse, (size_t)c->me_chunk * c->ne * c->nr);
  rc |= dev_alloc(&c->windows, (size_t)c->wy * 6 * c->ws);
  if (c->use_lds) rc |= dev_alloc(&c->wcell, 4 * (size_t)update_lds_float4s(c->wx, c->wy));
  rc |= dev_alloc(&c->dmat, (size_t)kBlockN * kBlockN);
  rc |= dev_alloc(&c->sd, (size_t)c->ne * c->max_obs * 2);
  rc |= dev_alloc(&c->vblk, (size_t)c->ne * std::max(1, c->max_obs) * kBlockN);
  rc |= dev_alloc(&c->pcoef, (size_t)3 * c->ne);
  rc |= dev_alloc(&c->sdf, (size_t)sd_float_stride(c->ne) * (c->max_obs + 1) * 2);
  // the padding particles' entries are read (and their sums dropped): keep them finite; row
  // max_obs stays zero
  if (rc == 0 && hipMemset(c->sdf, 0, sizeof(float) * sd_float_stride(c->ne) * (c->max_obs + 1) *
                                          2) != hipSuccess)
    rc = fail(IEWPF_E_HIP, "hipMemset(sdf)");
  rc |= dev_alloc(&c->cval, c->ne);
  rc |= dev_alloc(&c->dots, (size_t)3 * c->ne);
  rc |= dev_alloc(&c->part_dots, (size_t)3 * c->ne * rand_dots_parts());
  rc |= dev_alloc(&c->alpha, c->ne);
  rc |= dev_alloc(&c->cstar, c->ne);
  rc |= dev_alloc(&c->scal, 16);
  c->stage_bytes = stage_layout(*c).total;
  rc |= dev_alloc(&c->d_stage, c->stage_bytes);
  rc |= dev_alloc(&c->dk1, (size_t)c->ne * c->max_obs * 2);
  rc |= dev_alloc(&c->dpstar, (size_t)c->ne * c->max_obs * 2);
  rc |= dev_alloc(&c->dobs, (size_t)c->max_obs * 2);
  rc |= dev_alloc(&c->cflmax, 2);
  rc |= dev_alloc(&c->dparents, (size_t)c->ne);
  rc |= dev_alloc(&c->dcum, (size_t)c->ne);
  rc |= dev_alloc(&c->sir_parents, (size_t)c->ne);
  rc |= dev_alloc(&c->dobs_cells, (size_t)c->max_obs * 2);
  if (rc) {
    free_ctx(c);
    return IEWPF_E_HIP;
  }
  {
    const StageLayout L = stage_layout(*c);
    c->obs_cells = reinterpret_cast<int32_t*>(c->d_stage + L.cells);
    c->obs_y = reinterpret_cast<double*>(c->d_stage + L.y);
    c->pt_off = reinterpret_cast<int32_t*>(c->d_stage + L.pt_off);
    c->pt_ent = reinterpret_cast<int32_t*>(c->d_stage + L.pt_ent);
    c->st_off = reinterpret_cast<int32_t*>(c->d_stage + L.st_off);
    c->st_rows = reinterpret_cast<int32_t*>(c->d_stage + L.st_rows);
    c->st_ent = reinterpret_cast<int32_t*>(c->d_stage + L.st_ent);
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_stage), c->stage_bytes) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_sync), sizeof(double) * 16) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_small),
                    sizeof(double) * std::max<size_t>(64, std::max<size_t>(2 * c->max_obs, 8 * (size_t)c->ne))) !=
          hipSuccess ||
      hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming) != hipSuccess) {
    free_ctx(c);
    return fail(IEWPF_E_HIP, "pinned host allocation failed");
  }
  {
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, c->h_stage, 0) == hipSuccess)
      c->h_stage_dev = static_cast<unsigned char*>(dp);
  }
  c->h_win64 = win;
  // device layout [wy][6][ws]: the six fields of one window cell a fixed stride apart
  std::vector<float> winf((size_t)c->wy * 6 * c->ws, 0.0f);
  for (int fld = 0; fld < 6; ++fld)
    for (int iy = 0; iy < c->wy; ++iy)
      for (int ix = 0; ix < c->wx; ++ix)
        winf[((size_t)iy * 6 + fld) * c->ws + ix] =
            (float)win[((size_t)fld * c->wy + iy) * c->wx + ix];
  // cell-major copy staged in LDS by the update: the cells, one zero cell, zero padding
  std::vector<float> wcf(c->wcell ? 4 * (size_t)update_lds_float4s(c->wx, c->wy) : 0, 0.0f);
  if (c->wcell)
    for (int fld = 0; fld < 6; ++fld)
      for (int iy = 0; iy < c->wy; ++iy)
        for (int ix = 0; ix < c->wx; ++ix)
          wcf[((size_t)iy * c->wx + ix) * 6 + fld] =
              (float)win[((size_t)fld * c->wy + iy) * c->wx + ix];
  std::vector<float> dm((size_t)kBlockN * kBlockN);
  for (int i = 0; i < kBlockN; ++i)
    for (int j = 0; j < kBlockN; ++j)
      dm[i * kBlockN + j] = (float)(c->ahalf[i * kBlockN + j] - (i == j ? 1.0 : 0.0));
  if (hipMemcpy(c->windows, winf.data(), sizeof(float) * winf.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      (c->wcell && hipMemcpy(c->wcell, wcf.data(), sizeof(float) * wcf.size(),
                             hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(c->dmat, dm.data(), sizeof(float) * dm.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_ctx(c);
    return fail(IEWPF_E_HIP, "constant upload failed");
  }
  *out = c;
  return 0;
}

void iewpf_destroy(iewpf_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  free_ctx(ctx);
}

int iewpf_window_size(iewpf_ctx* ctx, int32_t* wx, int32_t* wy) {
  if (!ctx || !wx || !wy) return fail(IEWPF_E_ARG, "NULL argument");
  *wx = ctx->wx;
  *wy = ctx->wy;
  return 0;
}

int iewpf_init_ensemble(iewpf_ctx* c, float* state, const float* base, uint64_t stream_index,
                        void* stream) {
  if (!c || !state) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  if (!base) IEWPF_HIP_TRY(hipMemsetAsync(state, 0, sizeof(float) * 3 * c->ncell * c->ne, s));
  launch_normals(c->xi, c->nr, c->ne, c->cfg.seed, stream_index, kTagInit, c->cfg.ensemble_id, s);
  launch_soar(c->cc, c->soar_init_f, c->ne, c->xi, c->coarse, s);
  launch_gb_add(c->cc, c->ne, c->coarse, base, state, c->gb_strip_h, s);
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_step_ensemble(iewpf_ctx* c, float* state, int n_model_steps, uint64_t first_step,
                        int noise_on_last, void* stream) {
  if (!c || !state || n_model_steps < 0) return fail(IEWPF_E_ARG, "invalid argument");
  return model_steps(c, state, n_model_steps, first_step, noise_on_last, as_stream(stream));
}

int iewpf_perturb(iewpf_ctx* c, float* state, uint64_t step_index, void* stream) {
  if (!c || !state) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  add_noise(c, state, step_index, s);
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_set_scheme(iewpf_ctx* c, int scheme) {
  if (!c || scheme < 0 || scheme > 2) return fail(IEWPF_E_ARG, "scheme must be 0, 1 or 2");
  if (scheme == 2 && (3 * c->ncell) % 4 != 0)
    return fail(IEWPF_E_SHAPE, "3 nx ny must be a multiple of 4 for the particle gather");
  c->one_stage = scheme == 1;
  c->sir = scheme == 2;
  return 0;
}

int iewpf_set_full_innovation(iewpf_ctx* c, int on) {
  if (!c) return fail(IEWPF_E_ARG, "NULL context");
  if (!on) {
    c->full_innov = false;
    return 0;
  }
  const int n = 2 * c->max_obs;
  if (n > chol_max_order()) return fail(IEWPF_E_CAPACITY, "2 max_obs exceeds the full-covariance limit");
  if (!c->fS) {
    int rc = 0;
    rc |= dev_alloc(&c->windows64, c->h_win64.size());
    rc |= dev_alloc(&c->fS, (size_t)n * n);
    rc |= dev_alloc(&c->fX, (size_t)n * n);
    rc |= dev_alloc(&c->dinn, (size_t)c->ne * c->max_obs * 2);
    rc |= dev_alloc(&c->fstatus, 1);
    if (rc) return IEWPF_E_HIP;
    IEWPF_HIP_TRY(hipMemcpy(c->windows64, c->h_win64.data(), sizeof(double) * c->h_win64.size(),
                            hipMemcpyHostToDevice));
  }
  c->full_innov = true;
  c->f_n = -1;
  return 0;
}

int iewpf_assimilate(iewpf_ctx* c, float* state, const iewpf_obs* obs, int n_obs,
                     uint64_t analysis_index, iewpf_stats* stats_out, void* stream) {
  if (!c || !state || (n_obs > 0 && !obs) || n_obs < 0) return fail(IEWPF_E_ARG, "invalid argument");
  if (n_obs > c->max_obs) return fail(IEWPF_E_CAPACITY, "more observations than max_obs");
  hipStream_t s = as_stream(stream);
  if (int rc = wait_stage(c)) return rc;
  const StageLayout L = stage_layout(*c);
  int32_t* cells = reinterpret_cast<int32_t*>(c->h_stage + L.cells);
  double* y = reinterpret_cast<double*>(c->h_stage + L.y);
  for (int o = 0; o < n_obs; ++o) {
    cells[2 * o] = obs[o].j;
    cells[2 * o + 1] = obs[o].k;
    y[2 * o] = obs[o].y_hu;
    y[2 * o + 1] = obs[o].y_hv;
  }
  if (int rc = check_cells(c, cells, n_obs)) return rc;
  // unchanged cells: the kernels read y from the pinned staging area (this call waits for
  // them before it returns, so the host writes it again only after they are done)
  if (int rc = upload_observations(c, n_obs, true, s, true)) return rc;
  int rc_launch = 0;
  if (c->full_innov && !c->sir && n_obs > 0) rc_launch = prepare_full_s(c, cells, n_obs, s);
  // the sync kernel publishes the scalars and status words to mapped host memory (the SIR
  // path has no sync kernel: one copy back instead)
  c->publish_host = !c->sir;
  if (rc_launch == 0) rc_launch = launch_analysis(c, state, n_obs, analysis_index, nullptr, s);
  c->publish_host = false;
  if (rc_launch) {
    (void)hipStreamSynchronize(s);  // nothing may still read the staging area
    c->y_use = nullptr;
    return rc_launch;
  }
  const double* v = c->h_sync;
  if (c->sir) {
    IEWPF_HIP_TRY(hipMemcpyAsync(c->h_small, c->scal, sizeof(double) * (kScalStatus + 2),
                                 hipMemcpyDeviceToHost, s));
    v = c->h_small;
  }
  const hipError_t es = hipStreamSynchronize(s);
  c->y_use = nullptr;
  IEWPF_HIP_TRY(es);
  if (!c->sir && reinterpret_cast<const int32_t*>(c->h_sync + kScalStatus)[4] != 0) {
    // the update found a non-finite value: its status words are on the device
    IEWPF_HIP_TRY(hipMemcpy(c->h_sync + kScalStatus + 1, c->scal + kScalStatus + 1,
                            sizeof(double), hipMemcpyDeviceToHost));
  }
  if (stats_out) {
    stats_out->cbar = v[0];
    stats_out->beta = v[1];
    stats_out->alpha_min = v[2];
    stats_out->alpha_max = v[3];
    stats_out->cstar_max = v[4];
    stats_out->c_min = v[5];
    stats_out->c_max = v[6];
    stats_out->argmin_beta = (int32_t)v[7];
    stats_out->n_obs = n_obs;
  }
  return analysis_status(reinterpret_cast<const int32_t*>(v + kScalStatus), "");
}

int iewpf_particle_scalars(iewpf_ctx* c, double* out, void* stream) {
  if (!c || !out) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  std::vector<double> cv(c->ne), dt(3 * (size_t)c->ne), al(c->ne), cs(c->ne);
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  IEWPF_HIP_TRY(hipMemcpy(cv.data(), c->cval, sizeof(double) * c->ne, hipMemcpyDeviceToHost));
  IEWPF_HIP_TRY(hipMemcpy(dt.data(), c->dots, sizeof(double) * 3 * c->ne, hipMemcpyDeviceToHost));
  IEWPF_HIP_TRY(hipMemcpy(al.data(), c->alpha, sizeof(double) * c->ne, hipMemcpyDeviceToHost));
  IEWPF_HIP_TRY(hipMemcpy(cs.data(), c->cstar, sizeof(double) * c->ne, hipMemcpyDeviceToHost));
  const double scale = c->n_psi / (double)c->nr;
  for (int i = 0; i < c->ne; ++i) {
    double* o = out + 8 * (size_t)i;
    o[0] = cv[i];
    o[1] = dt[3 * i] * scale;
    o[2] = dt[3 * i + 1] * scale;
    o[3] = al[i];
    o[4] = cs[i];
    o[5] = dt[3 * i];
    o[6] = dt[3 * i + 1];
    o[7] = dt[3 * i + 2];
  }
  return 0;
}

int iewpf_observe_moorings(iewpf_ctx* c, const float* truth, const int32_t* cells_host, int n_obs,
                           uint64_t analysis_index, iewpf_obs* obs_host, void* stream) {
  if (!c || !truth || !cells_host || !obs_host || n_obs < 0) return fail(IEWPF_E_ARG, "NULL argument");
  if (n_obs > c->max_obs) return fail(IEWPF_E_CAPACITY, "more observations than max_obs");
  if (int rc = check_cells(c, cells_host, n_obs)) return rc;
  if (n_obs == 0) return 0;
  hipStream_t s = as_stream(stream);
  if (int rc = wait_stage(c)) return rc;
  const StageLayout L = stage_layout(*c);
  int32_t* cells = reinterpret_cast<int32_t*>(c->h_stage + L.cells);
  std::memcpy(cells, cells_host, sizeof(int32_t) * 2 * n_obs);
  c->list_n = -1;  // the device cells no longer match the device lists
  IEWPF_HIP_TRY(hipMemcpyAsync(c->obs_cells, cells, sizeof(int32_t) * 2 * n_obs,
                               hipMemcpyHostToDevice, s));
  launch_observe(n_obs, c->nx, c->ny, c->cfg.H, c->cfg.obs_sigma, c->cfg.seed, analysis_index,
                 c->cfg.ensemble_id, truth, c->obs_cells, c->dobs, s);
  IEWPF_HIP_TRY(hipGetLastError());
  IEWPF_HIP_TRY(hipMemcpyAsync(c->h_small, c->dobs, sizeof(double) * 2 * n_obs,
                               hipMemcpyDeviceToHost, s));
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  for (int o = 0; o < n_obs; ++o) {
    obs_host[o].j = cells_host[2 * o];
    obs_host[o].k = cells_host[2 * o + 1];
    obs_host[o].y_hu = c->h_small[2 * o];
    obs_host[o].y_hv = c->h_small[2 * o + 1];
  }
  return 0;
}

int iewpf_observe_drifters(iewpf_ctx* c, const double* pos_now, const double* pos_prev, int n,
                           double dt_obs, uint64_t analysis_index, iewpf_obs* obs_host,
                           void* stream) {
  if (!c || !pos_now || !pos_prev || !obs_host || n < 0 || !(dt_obs > 0))
    return fail(IEWPF_E_ARG, "invalid argument");
  if (n > c->max_obs) return fail(IEWPF_E_CAPACITY, "more drifters than max_obs");
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  const auto& f = c->cfg;
  launch_observe_drifters(n, c->nx, c->ny, f.dx, f.dy, f.H, f.obs_sigma, dt_obs, f.seed,
                          analysis_index, f.ensemble_id, pos_now, pos_prev, c->dobs_cells, c->dobs, s);
  IEWPF_HIP_TRY(hipGetLastError());
  // y then the cells, one pinned buffer (h_small holds at least 2 max_obs doubles; the cells
  // take max_obs more)
  std::vector<int32_t> cells(2 * (size_t)n);
  IEWPF_HIP_TRY(hipMemcpyAsync(c->h_small, c->dobs, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s));
  IEWPF_HIP_TRY(hipMemcpyAsync(cells.data(), c->dobs_cells, sizeof(int32_t) * 2 * n,
                               hipMemcpyDeviceToHost, s));
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  for (int d = 0; d < n; ++d) {
    obs_host[d].j = cells[2 * d];
    obs_host[d].k = cells[2 * d + 1];
    obs_host[d].y_hu = c->h_small[2 * d];
    obs_host[d].y_hv = c->h_small[2 * d + 1];
  }
  return 0;
}

int iewpf_sir_log_weights(iewpf_ctx* c, const float* state, const iewpf_obs* obs, int n_obs,
                          double r_scale, double* logw, double* w_out, void* stream) {
  if (!c || !state || !logw || (n_obs > 0 && !obs) || n_obs < 0 || !(r_scale > 0))
    return fail(IEWPF_E_ARG, "invalid argument");
  if (n_obs > c->max_obs) return fail(IEWPF_E_CAPACITY, "more observations than max_obs");
  hipStream_t s = as_stream(stream);
  if (int rc = wait_stage(c)) return rc;
  const StageLayout L = stage_layout(*c);
  int32_t* cells = reinterpret_cast<int32_t*>(c->h_stage + L.cells);
  double* y = reinterpret_cast<double*>(c->h_stage + L.y);
  for (int o = 0; o < n_obs; ++o) {
    cells[2 * o] = obs[o].j;
    cells[2 * o + 1] = obs[o].k;
    y[2 * o] = obs[o].y_hu;
    y[2 * o + 1] = obs[o].y_hv;
  }
  if (int rc = check_cells(c, cells, n_obs)) return rc;
  // cells and values only: the device lists no longer match the device cells
  c->list_n = -1;
  if (n_obs > 0)
    IEWPF_HIP_TRY(hipMemcpyAsync(c->d_stage, c->h_stage, L.y + sizeof(double) * 2 * n_obs,
                                 hipMemcpyHostToDevice, s));
  IEWPF_HIP_TRY(hipEventRecord(c->stage_ev, s));
  c->stage_pending = true;
  const double r = r_scale * c->cfg.obs_sigma * c->cfg.obs_sigma;
  const double Rinv[4] = {1.0 / r, 0.0, 0.0, 1.0 / r};
  launch_innovation(c->ne, n_obs, c->max_obs, c->nx, c->ny, c->cfg.H, Rinv, state, c->obs_cells,
                    c->obs_y, c->sd, nullptr, logw, s, -0.5);
  if (w_out) launch_sir_normalise(c->ne, logw, w_out, s);
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_advect_drifters(iewpf_ctx* c, const float* psi_n, const float* psi_np1, double* pos,
                          int n_drifters, void* stream) {
  if (!c || !psi_n || !psi_np1 || !pos || n_drifters < 0) return fail(IEWPF_E_ARG, "NULL argument");
  if (n_drifters > c->max_obs) return fail(IEWPF_E_CAPACITY, "more drifters than max_obs");
  if (n_drifters == 0) return 0;
  hipStream_t s = as_stream(stream);
  const auto& f = c->cfg;
  launch_drift_k1(c->ne, n_drifters, c->nx, c->ny, f.dx, f.dy, f.H, f.dt, psi_n, pos, c->dk1,
                  c->dpstar, s);
  launch_drift_k2(c->ne, n_drifters, c->nx, c->ny, f.dx, f.dy, f.H, f.dt, psi_np1, pos, c->dk1,
                  c->dpstar, nullptr, s);
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_forecast_drifters(iewpf_ctx* c, float* state, double* pos, int n_drifters,
                            int n_model_steps, uint64_t first_step, double* traj, void* stream) {
  if (!c || !state || !pos || n_drifters < 0 || n_model_steps < 0)
    return fail(IEWPF_E_ARG, "invalid argument");
  if (n_drifters > c->max_obs) return fail(IEWPF_E_CAPACITY, "more drifters than max_obs");
  hipStream_t s = as_stream(stream);
  const auto& f = c->cfg;
  const size_t per = (size_t)c->ne * n_drifters * 2;
  if (traj && per)
    IEWPF_HIP_TRY(hipMemcpyAsync(traj, pos, sizeof(double) * per, hipMemcpyDeviceToDevice, s));
  for (int st = 0; st < n_model_steps; ++st) {
    if (n_drifters)
      launch_drift_k1(c->ne, n_drifters, c->nx, c->ny, f.dx, f.dy, f.H, f.dt, state, pos, c->dk1,
                      c->dpstar, s);
    if (int rc = model_steps(c, state, 1, first_step + st, 1, s)) return rc;
    if (n_drifters)
      launch_drift_k2(c->ne, n_drifters, c->nx, c->ny, f.dx, f.dy, f.H, f.dt, state, pos, c->dk1,
                      c->dpstar, traj ? traj + (size_t)(st + 1) * per : nullptr, s);
  }
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_resample(iewpf_ctx* c, float* state, const double* logw, uint64_t analysis_index,
                   int32_t* parents, void* stream) {
  if (!c || !state || !logw || !parents) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  launch_resample(c->ne, c->cfg.seed, analysis_index, c->cfg.ensemble_id, logw, parents,
                  c->dparents, c->dcum, s);
  const size_t per = 3 * c->ncell;
  if (per % 4 == 0) {
    launch_gather_particles(c->ne, per, parents, state, c->scratch, s);
  } else {
    return fail(IEWPF_E_SHAPE, "3 nx ny must be a multiple of 4 for the particle gather");
  }
  IEWPF_HIP_TRY(hipMemcpyAsync(state, c->scratch, sizeof(float) * per * c->ne,
                               hipMemcpyDeviceToDevice, s));
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}


int iewpf_autotune(iewpf_ctx* c, const float* state, int32_t* strip_out, void* stream) {
  if (!c || !state || !strip_out) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  // the strip form (batched launches use it) and, when the context runs the full-row form,
  // that form too
  SweConst best;
  if (int rc = tune_strip(c, c->swe_halo, state, s, &best)) return rc;
  c->swe_halo = best;
  if (c->swe.row) {
    if (int rc = tune_strip(c, c->swe, state, s, &best)) return rc;
    c->swe = best;
  } else {
    c->swe = c->swe_halo;
  }
  *strip_out = c->swe.strip_h;
  return 0;
}

int iewpf_set_strip_rows(iewpf_ctx* c, int rows) {
  if (!c || rows < 1) return fail(IEWPF_E_ARG, "strip rows must be >= 1");
  for (SweConst* C : {&c->swe, &c->swe_halo}) {
    C->strip_h = std::min(rows, c->ny);
    C->n_strip_y = (c->ny + C->strip_h - 1) / C->strip_h;
  }
  return 0;
}

int iewpf_batch_create(iewpf_ctx* const* ctxs, float* const* states, int n, iewpf_batch** out) {
  if (!ctxs || !states || !out || n <= 0 || n > kMaxBatch) return fail(IEWPF_E_ARG, "invalid argument");
  *out = nullptr;
  for (int e = 0; e < n; ++e) {
    if (!ctxs[e] || !states[e]) return fail(IEWPF_E_ARG, "NULL context or state");
    if (ctxs[e]->cfg.n_sub != ctxs[0]->cfg.n_sub || ctxs[e]->cfg.dt != ctxs[0]->cfg.dt)
      return fail(IEWPF_E_ARG, "batched ensembles need the same dt and n_sub");
    if (ctxs[e]->full_innov)
      return fail(IEWPF_E_ARG, "batched cycles use the independent-block innovation covariance");
    if (ctxs[e]->sir) return fail(IEWPF_E_ARG, "batched cycles run the IEWPF, not the SIR filter");
  }
  iewpf_batch* b = new iewpf_batch();
  b->n = n;
  b->n_sub = ctxs[0]->cfg.n_sub;
  b->split = env_int("IEWPF_BATCH_SPLIT", 1) != 0;
  SweJobTable plain{}, noise{};
  plain.n = noise.n = n;
  int w = 0;
  size_t ylen = 0;
  for (int e = 0; e < n; ++e) {
    iewpf_ctx* c = ctxs[e];
    b->ctx.push_back(c);
    b->state.push_back(states[e]);
    b->n_obs.push_back(0);
    b->y_off.push_back(ylen);
    ylen += 2 * (size_t)c->max_obs;
    SweJob J{};
    J.C = c->swe_halo;
    J.z = nullptr;
    J.z_field = 0;
    J.buf_a = states[e];
    J.buf_b = c->scratch;
    J.wave_begin = w;
    plain.job[e] = J;
    J.z = c->me_coarse;
    J.z_field = (size_t)c->ne * c->nr;
    noise.job[e] = J;
    w += c->ne * c->swe_halo.n_strip_x * c->swe_halo.n_strip_y;
  }
  plain.total_waves = noise.total_waves = w;
  b->total_waves = w;
  b->h_y_len = ylen;
  bool ok = hipMalloc(reinterpret_cast<void**>(&b->tab_plain), sizeof(SweJobTable)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->tab_noise), sizeof(SweJobTable)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_dyn), 2 * sizeof(uint64_t)) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_dyn), 2 * sizeof(uint64_t)) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_y), sizeof(double) * std::max<size_t>(ylen, 1)) ==
                hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_status), sizeof(int32_t) * 4 * n) == hipSuccess &&
            hipEventCreateWithFlags(&b->copy_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->in_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->out_ev, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking) == hipSuccess &&
            [&] {
              const int n_side = std::max(1, std::min(n, env_int("IEWPF_BATCH_STREAMS", 8)));
              for (int i = 0; i < n_side; ++i) {
                hipStream_t x = nullptr;
                if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) return false;
                b->side.push_back(x);
              }
              return true;
            }() &&
            hipMemcpy(b->tab_plain, &plain, sizeof(SweJobTable), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(b->tab_noise, &noise, sizeof(SweJobTable), hipMemcpyHostToDevice) == hipSuccess &&
            [&] {
              void* py = nullptr;
              void* pd = nullptr;
              void* ps = nullptr;
              if (hipHostGetDevicePointer(&py, b->h_y, 0) != hipSuccess ||
                  hipHostGetDevicePointer(&pd, b->h_dyn, 0) != hipSuccess ||
                  hipHostGetDevicePointer(&ps, b->h_status, 0) != hipSuccess)
                return false;
              b->h_y_dev = static_cast<const double*>(py);
              b->h_dyn_dev = static_cast<const uint64_t*>(pd);
              b->h_status_dev = static_cast<int32_t*>(ps);
              return true;
            }();
  if (!ok) {
    free_batch(b);
    return fail(IEWPF_E_HIP, "batch allocation failed");
  }
  *out = b;
  return 0;
}

void iewpf_batch_destroy(iewpf_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_batch(b);
}

int iewpf_batch_set_cells(iewpf_batch* b, int e, const int32_t* cells_host, int n_obs, void* stream) {
  if (!b || e < 0 || e >= b->n || (n_obs > 0 && !cells_host) || n_obs < 0)
    return fail(IEWPF_E_ARG, "invalid argument");
  iewpf_ctx* c = b->ctx[e];
  if (n_obs > c->max_obs) return fail(IEWPF_E_CAPACITY, "more observations than max_obs");
  if (int rc = check_cells(c, cells_host, n_obs)) return rc;
  hipStream_t s = as_stream(stream);
  if (int rc = wait_stage(c)) return rc;
  const StageLayout L = stage_layout(*c);
  std::memcpy(c->h_stage + L.cells, cells_host, sizeof(int32_t) * 2 * n_obs);
  if (int rc = upload_observations(c, n_obs, false, s)) return rc;
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  c->stage_pending = false;
  b->n_obs[e] = n_obs;
  if (b->exec) {  // observation lists changed: capture again
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = -1;
  }
  return 0;
}

int iewpf_batch_cycle(iewpf_batch* b, int n_model_steps, uint64_t first_step,
                      uint64_t analysis_index, const double* const* y_host, int use_graph,
                      void* stream) {
  if (!b || n_model_steps < 1 || !y_host) return fail(IEWPF_E_ARG, "invalid argument");
  hipStream_t s = as_stream(stream);
  hipStream_t run = use_graph ? b->gs : s;
  if (use_graph) {  // order the internal stream after the caller's work
    IEWPF_HIP_TRY(hipEventRecord(b->in_ev, s));
    IEWPF_HIP_TRY(hipStreamWaitEvent(run, b->in_ev, 0));
  }
  // observation values and counters into the pinned buffers the cycle's first kernel reads:
  // only once no earlier cycle can still read them (every cycle is waited for before this
  // call returns, except one that failed part-way, whose event is waited for here)
  for (int e = 0; e < b->n; ++e)
    if (b->n_obs[e] > 0 && !y_host[e]) return fail(IEWPF_E_ARG, "missing observation values");
  if (b->copy_pending) {
    IEWPF_HIP_TRY(hipEventSynchronize(b->copy_ev));
    b->copy_pending = false;
  }
  for (int e = 0; e < b->n; ++e)
    std::memcpy(b->h_y + b->y_off[e], y_host[e], sizeof(double) * 2 * b->n_obs[e]);
  b->h_dyn[0] = first_step;
  b->h_dyn[1] = analysis_index;
  if (!use_graph) {
    const int rc = batch_cycle_all(b, n_model_steps, first_step, analysis_index, false, s);
    IEWPF_HIP_TRY(hipEventRecord(b->copy_ev, s));
    b->copy_pending = true;
    if (rc) return rc;
    return batch_status(b, s);
  }

  if (!b->exec || b->graph_steps != n_model_steps) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
    }
    std::vector<bool> tr(b->n);
    for (int e = 0; e < b->n; ++e) {
      tr[e] = b->ctx[e]->trace;
      b->ctx[e]->trace = false;  // no event records inside a capture
    }
    IEWPF_HIP_TRY(hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal));
    const int rc = batch_cycle_all(b, n_model_steps, 0, 0, true, run);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(run, &g);
    for (int e = 0; e < b->n; ++e) b->ctx[e]->trace = tr[e];
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(IEWPF_E_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    b->graph = g;
    IEWPF_HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->graph_steps = n_model_steps;
  }
  IEWPF_HIP_TRY(hipGraphLaunch(b->exec, run));
  IEWPF_HIP_TRY(hipEventRecord(b->copy_ev, run));
  b->copy_pending = true;
  IEWPF_HIP_TRY(hipEventRecord(b->out_ev, run));
  IEWPF_HIP_TRY(hipStreamWaitEvent(s, b->out_ev, 0));
  return batch_status(b, run);
}

}  // extern "C"

namespace {
// The guarded window up to the drift flags: the inputs saved, the network applied (in as many
// particles at a time as its workspaces hold), each particle's relative mass drift and flag.
int window_forward(iewpf_ctx* c, iewpf_net* net, float* state, int n_model_steps,
                   double drift_tol, hipStream_t s) {
  if (!c || !net || !state || n_model_steps < 1 || !(drift_tol >= 0))
    return fail(IEWPF_E_ARG, "invalid argument");
  if (n_model_steps != net_horizon(net))
    return fail(IEWPF_E_ARG, "n_model_steps (" + std::to_string(n_model_steps) +
                                 ") differs from the network's horizon (" +
                                 std::to_string(net_horizon(net)) + " model steps)");
  const size_t per = 3 * c->ncell;
  // each buffer on its own, so a call after a failed allocation retries what is missing
  if (!c->saved) IEWPF_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&c->saved), sizeof(float) * per * c->ne));
  if (!c->sdrift) IEWPF_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&c->sdrift), sizeof(double) * c->ne));
  if (!c->sflags) IEWPF_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&c->sflags), sizeof(int32_t) * c->ne));
  IEWPF_HIP_TRY(hipMemcpyAsync(c->saved, state, sizeof(float) * per * c->ne, hipMemcpyDeviceToDevice, s));
  const int chunk = net_max_cells(net) / (int)std::min<size_t>(c->ncell, (size_t)INT32_MAX);
  if (chunk < 1) return fail(IEWPF_E_CAPACITY, "the network holds fewer cells than one particle");
  for (int p0 = 0; p0 < c->ne; p0 += chunk) {
    const int nb = std::min(chunk, c->ne - p0);
    if (int rc = iewpf_net_forward(net, c->saved + per * p0, state + per * p0, nb, c->ny, c->nx, s))
      return rc;
  }
  launch_mass_drift(c->saved, state, c->ne, (int)c->ncell, c->cfg.H, drift_tol, c->sdrift, c->sflags, s);
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}
}  // namespace

extern "C" {

int iewpf_surrogate_window(iewpf_ctx* c, iewpf_net* net, float* state, int n_model_steps,
                           uint64_t first_step, double drift_tol, double noise_scale,
                           int32_t* n_fallback_out, double* drift_out, void* stream) {
  if (!n_fallback_out) return fail(IEWPF_E_ARG, "invalid argument");
  hipStream_t s = as_stream(stream);
  if (int rc = window_forward(c, net, state, n_model_steps, drift_tol, s)) return rc;
  const size_t per = 3 * c->ncell;
  std::vector<int32_t> flags(c->ne);
  std::vector<double> drift(c->ne);
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  IEWPF_HIP_TRY(hipMemcpy(flags.data(), c->sflags, sizeof(int32_t) * c->ne, hipMemcpyDeviceToHost));
  IEWPF_HIP_TRY(hipMemcpy(drift.data(), c->sdrift, sizeof(double) * c->ne, hipMemcpyDeviceToHost));
  // Flagged particles: their saved inputs are packed into the scratch buffer and stepped
  // together by the plain scheme (deterministic model steps); the saved buffer, no longer
  // needed once packed, is the ping-pong partner.  Results are scattered back into state.
  std::vector<int> fl;
  for (int i = 0; i < c->ne; ++i)
    if (flags[i]) fl.push_back(i);
  const int nf = static_cast<int>(fl.size());
  if (nf > 0) {
    for (int k = 0; k < nf; ++k)
      IEWPF_HIP_TRY(hipMemcpyAsync(c->scratch + per * k, c->saved + per * fl[k], sizeof(float) * per,
                                   hipMemcpyDeviceToDevice, s));
    float* cur = c->scratch;
    float* other = c->saved;
    for (int st = 0; st < n_model_steps; ++st)
      for (int sub = 0; sub < c->cfg.n_sub; ++sub) {
        launch_swe_substep(c->swe, nf, cur, other, nullptr, s);
        std::swap(cur, other);
      }
    for (int k = 0; k < nf; ++k)
      IEWPF_HIP_TRY(hipMemcpyAsync(state + per * fl[k], cur + per * k, sizeof(float) * per,
                                   hipMemcpyDeviceToDevice, s));
  }
  if (noise_scale > 0.0) add_scaled_noise(c, state, first_step + n_model_steps - 1, noise_scale, s);
  IEWPF_HIP_TRY(hipGetLastError());
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  *n_fallback_out = nf;
  if (drift_out) std::memcpy(drift_out, drift.data(), sizeof(double) * c->ne);
  return 0;
}

int iewpf_surrogate_window_async(iewpf_ctx* c, iewpf_net* net, float* state, int n_model_steps,
                                 uint64_t first_step, double drift_tol, double noise_scale,
                                 int32_t* n_fallback_dev, double* drift_dev, void* stream) {
  if (!n_fallback_dev) return fail(IEWPF_E_ARG, "invalid argument");
  hipStream_t s = as_stream(stream);
  if (int rc = window_forward(c, net, state, n_model_steps, drift_tol, s)) return rc;
  const size_t per = 3 * c->ncell;
  // the flagged particles re-stepped in place from their saved inputs: every particle's
  // workgroups are launched and the unflagged ones return at once, so the host need not know
  // which particles drifted
  float* cur = c->saved;
  float* other = c->scratch;
  for (int st = 0; st < n_model_steps; ++st)
    for (int sub = 0; sub < c->cfg.n_sub; ++sub) {
      launch_swe_substep(c->swe, c->ne, cur, other, nullptr, s, c->sflags);
      std::swap(cur, other);
    }
  launch_copy_flagged(cur, state, c->sflags, c->ne, per, s);
  if (noise_scale > 0.0) add_scaled_noise(c, state, first_step + n_model_steps - 1, noise_scale, s);
  launch_count_flags(c->sflags, c->ne, n_fallback_dev, s);
  if (drift_dev)
    IEWPF_HIP_TRY(hipMemcpyAsync(drift_dev, c->sdrift, sizeof(double) * c->ne,
                                 hipMemcpyDeviceToDevice, s));
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_forecast_drifters_surrogate(iewpf_ctx* c, iewpf_net* net, float* state, double* pos,
                                      int n_drifters, int n_windows, int steps_per_window,
                                      uint64_t first_step, double drift_tol, double noise_scale,
                                      double* traj, int32_t* n_fallback_out, void* stream) {
  if (!c || !net || !state || !pos || n_drifters < 0 || n_windows < 0 || steps_per_window < 1)
    return fail(IEWPF_E_ARG, "invalid argument");
  if (n_drifters > c->max_obs) return fail(IEWPF_E_CAPACITY, "more drifters than max_obs");
  hipStream_t s = as_stream(stream);
  const auto& f = c->cfg;
  const size_t per_state = 3 * c->ncell * (size_t)c->ne;
  if (!c->wstart) IEWPF_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&c->wstart), sizeof(float) * per_state));
  const size_t per = (size_t)c->ne * n_drifters * 2;
  if (traj && per)
    IEWPF_HIP_TRY(hipMemcpyAsync(traj, pos, sizeof(double) * per, hipMemcpyDeviceToDevice, s));
  int total_fallback = 0;
  for (int w = 0; w < n_windows; ++w) {
    const uint64_t step0 = first_step + (uint64_t)w * steps_per_window;
    IEWPF_HIP_TRY(hipMemcpyAsync(c->wstart, state, sizeof(float) * per_state, hipMemcpyDeviceToDevice, s));
    int32_t nf = 0;
    if (int rc = iewpf_surrogate_window(c, net, state, steps_per_window, step0, drift_tol, 0.0, &nf,
                                        nullptr, stream))
      return rc;
    total_fallback += nf;
    // drifters: Heun steps in the states interpolated linearly in time across the window
    for (int st = 0; st < steps_per_window && n_drifters; ++st) {
      const double wa = (double)st / steps_per_window, wb = (double)(st + 1) / steps_per_window;
      launch_drift_k1(c->ne, n_drifters, c->nx, c->ny, f.dx, f.dy, f.H, f.dt, c->wstart, pos, c->dk1,
                      c->dpstar, s, state, wa);
      const size_t ti = (size_t)w * steps_per_window + st + 1;
      launch_drift_k2(c->ne, n_drifters, c->nx, c->ny, f.dx, f.dy, f.H, f.dt, c->wstart, pos, c->dk1,
                      c->dpstar, traj ? traj + ti * per : nullptr, s, state, wb);
    }
    if (noise_scale > 0.0) add_scaled_noise(c, state, step0 + steps_per_window - 1, noise_scale, s);
  }
  IEWPF_HIP_TRY(hipGetLastError());
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  if (n_fallback_out) *n_fallback_out = total_fallback;
  return 0;
}

int iewpf_check_cfl(iewpf_ctx* c, const float* state, double* dt_out, void* stream) {
  if (!c || !state || !dt_out) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  IEWPF_HIP_TRY(hipMemsetAsync(c->cflmax, 0, 2 * sizeof(unsigned), s));
  launch_cfl(c->ne, c->nx, c->ny, (float)c->cfg.H, (float)c->cfg.g, state, c->cflmax, s);
  IEWPF_HIP_TRY(hipGetLastError());
  unsigned w[2];
  IEWPF_HIP_TRY(hipMemcpyAsync(c->h_small, c->cflmax, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(w, c->h_small, sizeof(w));
  float sx, sy;
  std::memcpy(&sx, &w[0], 4);
  std::memcpy(&sy, &w[1], 4);
  const double dtc = 0.8 * 0.25 * std::min(c->cfg.dx / (double)sx, c->cfg.dy / (double)sy);
  *dt_out = dtc;
  if (!std::isfinite(dtc)) return fail(IEWPF_E_NONFINITE, "non-finite wave speed");
  if (c->cfg.dt / c->cfg.n_sub > dtc) return fail(IEWPF_E_CFL, "scheme step exceeds the CFL limit");
  return 0;
}

int iewpf_read_buffer(iewpf_ctx* c, int which, void* host_out, size_t bytes, void* stream) {
  if (!c || !host_out) return fail(IEWPF_E_ARG, "NULL argument");
  hipStream_t s = as_stream(stream);
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  const size_t nrf = sizeof(float) * (size_t)c->ne * c->nr;
  auto need = [&](size_t n) { return bytes == n; };
  switch (which) {
    case 0:
      if (!need(nrf)) break;
      IEWPF_HIP_TRY(hipMemcpy(host_out, c->xi, nrf, hipMemcpyDeviceToHost));
      return 0;
    case 1:
      if (!need(nrf)) break;
      IEWPF_HIP_TRY(hipMemcpy(host_out, c->nu, nrf, hipMemcpyDeviceToHost));
      return 0;
    case 2:
      if (!need(nrf)) break;
      IEWPF_HIP_TRY(hipMemcpy(host_out, c->coarse2, nrf, hipMemcpyDeviceToHost));
      return 0;
    case 3:
      if (!need(4 * sizeof(double))) break;
      std::memcpy(host_out, c->S, bytes);
      return 0;
    case 4:
      if (!need(4 * sizeof(double))) break;
      std::memcpy(host_out, c->Sc, bytes);
      return 0;
    case 5:
      if (!need(sizeof(double) * kBlockN * kBlockN)) break;
      std::memcpy(host_out, c->ahalf, bytes);
      return 0;
    case 6:
      if (!need(sizeof(float) * 6 * (size_t)c->wx * c->wy)) break;
      {
        std::vector<float> dev((size_t)c->wy * 6 * c->ws);
        IEWPF_HIP_TRY(hipMemcpy(dev.data(), c->windows, sizeof(float) * dev.size(),
                                hipMemcpyDeviceToHost));
        float* o = static_cast<float*>(host_out);
        for (int fld = 0; fld < 6; ++fld)
          for (int iy = 0; iy < c->wy; ++iy)
            for (int ix = 0; ix < c->wx; ++ix)
              o[((size_t)fld * c->wy + iy) * c->wx + ix] = dev[((size_t)iy * 6 + fld) * c->ws + ix];
      }
      return 0;
    case 7: {
      if (!need(sizeof(double) * (size_t)c->ne * c->last_n_obs * 2)) break;
      double* o = static_cast<double*>(host_out);
      for (int i = 0; i < c->ne; ++i)
        if (c->last_n_obs)
          IEWPF_HIP_TRY(hipMemcpy(o + (size_t)i * c->last_n_obs * 2, c->sd + (size_t)i * c->max_obs * 2,
                                  sizeof(double) * c->last_n_obs * 2, hipMemcpyDeviceToHost));
      return 0;
    }
    case 9: {
      const size_t n = 2 * (size_t)(c->f_n > 0 ? c->f_n : 0);
      if (!c->fX || n == 0 || !need(sizeof(double) * n * n)) break;
      IEWPF_HIP_TRY(hipMemcpy(host_out, c->fX, sizeof(double) * n * n, hipMemcpyDeviceToHost));
      return 0;
    }
    case 8:
      if (!need(25 * sizeof(double))) break;
      std::memcpy(host_out, c->soar_me, bytes);
      return 0;
    case 10:
      if (!need(sizeof(int32_t) * (size_t)c->ne)) break;
      IEWPF_HIP_TRY(hipMemcpy(host_out, c->sir_parents, bytes, hipMemcpyDeviceToHost));
      return 0;
    default:
      return fail(IEWPF_E_ARG, "unknown buffer id");
  }
  return fail(IEWPF_E_ARG, "byte count does not match the buffer");
}

}  // extern "C"
