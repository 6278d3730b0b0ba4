/*
 * iewpf.h -- C ABI of the MI355X (gfx950) IEWPF ensemble forecast + analysis library.
 *
 * Method: the two-stage implicit equal-weights particle filter applied to an ensemble of
 * rotating shallow-water models with SOAR-correlated, geostrophically balanced model
 * error (arXiv:1910.01031, Sections "The data-assimilation problem", "Simplified ocean
 * model for massively parallel architectures", "Efficient implementation of the IEWPF
 * scheme", Appendix A).
 *
 * Conventions shared by every call
 *   - State layout: float32, structure of arrays [n_particles][3][ny][nx], x fastest; the
 *     three fields are eta, hu, hv (eq. swe_full).  Cell (j, k) is centred at
 *     ((j + 1/2) dx, (k + 1/2) dy) (eq. cell_center); all boundaries are periodic.
 *   - Device pointers are plain HIP device pointers owned by the caller; `stream` is a
 *     hipStream_t passed as void* (NULL = the default stream).  Calls enqueue work on the
 *     stream and return without waiting unless stated otherwise.
 *   - Random numbers: counter-based Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 *     counter (block, step_or_analysis_index, (tag << 32) | ensemble_id, particle), four
 *     normals per block by Box-Muller in float64 (tags: model error 1, IEWPF xi 2,
 *     IEWPF nu 3, observation noise 4, initial state 5, resampling 6).  Results are a
 *     pure function of (config, indices, inputs): no atomics touch results.
 *   - Return value: 0 on success, a negative IEWPF_E_* code on failure (nothing is
 *     thrown across the ABI); iewpf_last_error() returns a thread-local message.
 *   - Host precompute (SOAR weights, pull windows, S, the local A^{1/2}) happens once in
 *     iewpf_create, which allocates the workspaces.  Later calls allocate device memory
 *     only where their description says so: the first call of an optional path (full
 *     innovation covariance, surrogate window, surrogate drifter forecast) and batch and
 *     network creation.
 *   - The context owns its constants and workspaces; calls on one context must not
 *     overlap in time (they share the workspaces).
 */
#ifndef IEWPF_H
#define IEWPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IEWPF_OK 0
#define IEWPF_E_ARG (-1)        /* invalid argument or NULL pointer                      */
#define IEWPF_E_SHAPE (-2)      /* grid not divisible by c_omega or < 7 coarse points      */
#define IEWPF_E_CFL (-3)        /* scheme step exceeds the CFL limit (eq. swecfl)          */
#define IEWPF_E_NONFINITE (-4)  /* non-finite value found in a particle                    */
#define IEWPF_E_BETA (-5)       /* beta <= 0: ensemble violates N_psi >> N_y (eq. betaTwoStage) */
#define IEWPF_E_HIP (-6)        /* a HIP runtime call failed                               */
#define IEWPF_E_CAPACITY (-7)   /* more observations/drifters than the context was built for */

typedef struct iewpf_ctx iewpf_ctx;

/* Grid, physics, model-error and filter constants of one ensemble.
 *   nx, ny, dx, dy     grid of nx x ny cells of dx x dy metres (eq. cell_center)
 *   H, g, f            equilibrium depth, gravity, Coriolis parameter (eq. swe_full)
 *   dt, n_sub          model step and its number of equal scheme steps (eq. swecfl)
 *   theta              generalized-minmod limiter parameter of the scheme (1 <= theta <= 2)
 *   c_omega            coarsening of the random grid Omega^R (Section "Small scale model errors"),
 *                      1 <= c_omega <= 16
 *   me_std, me_L0      model error: pointwise std of the coarse SOAR field and SOAR length
 *                      scale L0 (eq. soar_function); q0 = me_std / ||k||_2
 *   init_std, init_L0  same for the initial-state perturbation of iewpf_init_ensemble
 *   obs_sigma          observation error std, R = obs_sigma^2 I
 *   n_particles        ensemble size N_e, 1 .. 65535
 *   max_obs            capacity for observations / drifters per call
 *   seed, ensemble_id  Philox key word 0 and counter word 2 (low half)          */
typedef struct {
  int32_t nx, ny;
  double dx, dy, H, g, f, dt;
  int32_t n_sub;
  double theta;
  int32_t c_omega;
  double me_std, me_L0;
  double init_std, init_L0;
  double obs_sigma;
  int32_t n_particles;
  int32_t max_obs;
  uint64_t seed;
  uint32_t ensemble_id;
} iewpf_config;

/* One (hu, hv) observation in cell (j, k) (eq. stateObservation). */
typedef struct {
  int32_t j, k;
  double y_hu, y_hv;
} iewpf_obs;

/* Scalars of one analysis (Appendix A): cbar = w_target = mean c_i, beta, and ranges. */
typedef struct {
  double cbar, beta;
  double alpha_min, alpha_max;
  double cstar_max;
  double c_min, c_max;
  int32_t argmin_beta;
  int32_t n_obs;
} iewpf_stats;

/* Create a context: validates the config (c_omega <= 16, nx, ny divisible by c_omega, >= 7
 * coarse points per direction, nx ny < 178,956,970 cells per particle, obs/drifter
 * capacity; IEWPF_E_SHAPE for the grid limits), computes in float64 on the host the SOAR stencils,
 * the pull windows Q^{1/2} Q^{1/2,T} H^T e_b (eq. detailedOPDUpdate), S = (H Q H^T + R)^-1
 * by Cholesky (eq. S_extended), the local 49x49 A^{1/2} (eq. svdOfParenthesis), uploads
 * them and allocates the workspaces (one state-sized scratch buffer, coarse fields, and the
 * model-error fields of up to 16 model steps drawn ahead, about 64 MB at most).
 * *out receives the context; destroy with iewpf_destroy.  Uses the current HIP device. */
int iewpf_create(const iewpf_config* cfg, iewpf_ctx** out);
void iewpf_destroy(iewpf_ctx* ctx);

/* Initial ensemble (Section "Small scale model errors" applied with the init_* constants):
 * state[i] = base + Q_init^{1/2} xi_i, xi_i from stream (stream_index, tag 5, particle i).
 * base: device [3][ny][nx] or NULL (zero).  state: device [n_particles][3][ny][nx]. */
int iewpf_init_ensemble(iewpf_ctx* ctx, float* state, const float* base, uint64_t stream_index,
                        void* stream);

/* n_model_steps stochastic model steps (eq. model_equation): each is n_sub SSP-RK2 scheme
 * steps followed by the model error beta = Q^{1/2} xi with xi from stream (first_step + s,
 * tag 1); when noise_on_last is 0 the error is not added after the last step (the
 * forecast into an observation time is deterministic, Section "Observations and
 * innovations").  In place on state. */
int iewpf_step_ensemble(iewpf_ctx* ctx, float* state, int n_model_steps, uint64_t first_step,
                        int noise_on_last, void* stream);

/* Add one model-error draw (stream step_index, tag 1) to every particle, in place. */
int iewpf_perturb(iewpf_ctx* ctx, float* state, uint64_t step_index, void* stream);

/* Filter scheme of iewpf_assimilate: 0 (default) the two-stage IEWPF (target weight = mean
 * c_i, beta from eq. betaTwoStage, update eq. optUpdateEquationTwoStage); 1 the original
 * one-stage IEWPF of Appendix A (eq. iewpfUpdateAgain: no nu term; target weight
 * max_i c_i, eq. iewpf_targetWeight; c*_i = target - c_i, eq. iewpfCStar; alpha_i by eq.
 * iewpfAlphaSol).  With 1, stats_out->cbar is the target weight, beta is 0 and argmin_beta
 * is the particle with the largest c_i.  2 the standard particle filter (Section "Standard
 * particle filter"): log-weights l_i = -1/2 sum_o d^T R^{-1} d from the eta-compensated
 * innovations (eq. standardParticleFilterWeight), residual resampling with uniforms from
 * stream (analysis_index, tag 6) and the parents' states copied in (their indices: buffer 10
 * of iewpf_read_buffer); stats_out then has c_min / c_max = the range of -2 l_i,
 * argmin_beta = the particle of largest weight and the IEWPF fields 0; a non-finite l_i
 * leaves the state untouched and returns IEWPF_E_NONFINITE.  Scheme 2 needs 3 nx ny to be a
 * multiple of 4 (IEWPF_E_SHAPE) and is not available to batches.  A batch's graph keeps the
 * scheme its contexts had at its first cycle. */
int iewpf_set_scheme(iewpf_ctx* ctx, int scheme);

/* Full innovation covariance on (1) or off (0, the default).  The paper treats observations
 * independently: S = (H Q H^T + R)^{-1} is the same 2x2 block for every observation (eq.
 * S_extended and the assumption after it that observations are far apart).  When on,
 * iewpf_assimilate uses S = (sym(H Q H^T) + R)^{-1} over all observations together
 * ([2 n_obs]^2, float64 Cholesky on the device, S formed from the factor by triangular
 * solves of the unit vectors, then S d and c_i by one float64 product per analysis) in the
 * pull and in c_i; the posterior
 * perturbation keeps the paper's local blocks.  H Q H^T's entries are the pull windows read
 * at the offsets between observed cells; with c_Omega > 1 each observation's chain uses a
 * coarse grid aligned on its own cell, so its symmetric part is used.  The factor is rebuilt
 * only when the observed cells change (that call waits for the stream).  Requires
 * 2 max_obs <= 1024 (IEWPF_E_CAPACITY otherwise); allocates its buffers on the first call;
 * not available to batched cycles. */
int iewpf_set_full_innovation(iewpf_ctx* ctx, int on);

/* Two-stage IEWPF analysis of the forecast ensemble in place (Section "Efficient
 * implementation of the IEWPF scheme"): innovations, pull, perpendicular xi/nu (streams
 * (analysis_index, tags 2 and 3)), beta, alpha (Lambert W_0), local P^{1/2} and the
 * posterior update.  obs_host: n_obs host records (copied; the pointer may be reused
 * when the call returns).  The per-call observation index lists are built on the host
 * and uploaded with the values in one copy; when the cells equal the previous call's
 * (moorings), nothing is uploaded: the kernels read the values from the library's pinned,
 * device-mapped staging area (the call waits for them).  stats_out: host pointer or NULL
 * (filled when non-NULL).  The call waits for the analysis to finish and checks its status words:
 *   IEWPF_E_BETA       beta <= 0 (eq. betaTwoStage: the ensemble violates N_psi >> N_y);
 *                      the state is left untouched (stats_out still holds beta)
 *   IEWPF_E_NONFINITE  a non-finite c_i, gamma_i, zeta_i, c*_i or alpha_i (the state is left
 *                      untouched), or a non-finite value in an updated particle (the state
 *                      is updated; the message names the first such particle). */
int iewpf_assimilate(iewpf_ctx* ctx, float* state, const iewpf_obs* obs_host, int n_obs,
                     uint64_t analysis_index, iewpf_stats* stats_out, void* stream);

/* Per-particle scalars of the last analysis, copied to host after a stream sync:
 * out[i*8 + {0..7}] = c_i, gamma_i, zeta_i, alpha_i, c*_i, xi.xi, nu~.nu~, nu~.xi. */
int iewpf_particle_scalars(iewpf_ctx* ctx, double* out, void* stream);

/* Mooring observations of a truth state (eq. buoyObservation): for each cell (j, k) of
 * cells_host [2*n_obs], y = (hu, hv) H / (H + eta) + obs_sigma * n, n from stream
 * (analysis_index, tag 4, ensemble_id, particle 0), normals 2o and 2o+1.  truth: device
 * [3][ny][nx].  Writes n_obs records to obs_host (waits for the stream). */
int iewpf_observe_moorings(iewpf_ctx* ctx, const float* truth, const int32_t* cells_host,
                           int n_obs, uint64_t analysis_index, iewpf_obs* obs_host,
                           void* stream);

/* Drifter observations of a truth run (eq. drifterObservation): drifter d at unwrapped
 * positions pos_prev and pos_now (device float64 [n][2], metres) at two observation times
 * dt_obs seconds apart observes y_d = (pos_now - pos_prev) / dt_obs * H + obs_sigma * n, n from
 * stream (analysis_index, tag 4, ensemble_id, particle word 1), normals 2d and 2d+1; its
 * observed cell is (floor(x/dx) mod nx, floor(y/dy) mod ny) of pos_now (eq.
 * stateObservation).  Writes n records to obs_host (waits for the stream).  n <= max_obs
 * (IEWPF_E_CAPACITY), dt_obs > 0. */
int iewpf_observe_drifters(iewpf_ctx* ctx, const double* pos_now, const double* pos_prev, int n,
                           double dt_obs, uint64_t analysis_index, iewpf_obs* obs_host,
                           void* stream);

/* Log-weights of the standard particle filter (Section "Standard particle filter", eq.
 * standardParticleFilterWeight): l_i = -1/2 sum_o d_io^T R^{-1} d_io with the eta-compensated
 * innovations d (eq. etaCompensatedInnovation) and R = r_scale obs_sigma^2 I, float64.
 * logw: device float64 [n_particles]; w_out: device float64 [n_particles] or NULL, the
 * normalised weights exp(l_i - max l) / sum_j exp(l_j - max l).  obs_host is copied (n_obs <=
 * max_obs).  Feeds iewpf_resample. */
int iewpf_sir_log_weights(iewpf_ctx* ctx, const float* state, const iewpf_obs* obs_host, int n_obs,
                          double r_scale, double* logw, double* w_out, void* stream);

/* Drifter forecast: n_model_steps stochastic model steps (model error after every step,
 * stream first_step + s) while n_drifters drifters per particle are advected by Heun's
 * method with bilinear velocity u = (hu, hv)/(H + eta) from psi^n and psi^{n+1}.
 * pos: device float64 [n_particles][n_drifters][2] unwrapped metres, updated in place;
 * traj: device float64 [n_model_steps + 1][n_particles][n_drifters][2] or NULL. */
int iewpf_forecast_drifters(iewpf_ctx* ctx, float* state, double* pos, int n_drifters,
                            int n_model_steps, uint64_t first_step, double* traj, void* stream);

/* Advect drifters over one model step between two given states (no model stepping):
 * pos += dt/2 (u(pos; psi_n) + u(pos + dt u(pos; psi_n); psi_np1)). */
int iewpf_advect_drifters(iewpf_ctx* ctx, const float* psi_n, const float* psi_np1, double* pos,
                          int n_drifters, void* stream);

/* SIR residual resampling (Section "Standard particle filter"): from natural log-weights
 * logw (device float64 [n_particles]) draw parents (device int32 [n_particles], ascending)
 * with uniforms from stream (analysis_index, tag 6) and copy the parent states into state
 * (in place, via the context's scratch buffer). */
int iewpf_resample(iewpf_ctx* ctx, float* state, const double* logw, uint64_t analysis_index,
                   int32_t* parents, void* stream);

/* Residual resampling for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same draws,
 * parents and copies as iewpf_resample without a context, out of place, with its partial
 * results (floor counts, cumulative residuals) in a fixed device array of the library
 * (768 KiB per GPU, held until the process ends; its address is looked up once per device).
 * The call allocates nothing and does not wait.
 *   n_particles          1 .. 65535 (the array's size; IEWPF_E_CAPACITY above)
 *   floats_per_particle  floats of one particle's state (3 nx ny), a multiple of 4
 *                        (IEWPF_E_SHAPE otherwise)
 *   seed, ensemble_id    the Philox key word 0 and counter word 2 of iewpf_config
 *   logw                 device float64 [n_particles] natural log-weights
 *   state_in, state_out  device float32 [n_particles][floats_per_particle]; must not overlap
 *                        (IEWPF_E_ARG); state_out[i] = state_in[parents[i]]
 *   parents              device int32 [n_particles], ascending
 * Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (on
 * different streams or threads) race and must be serialised by the caller. */
int iewpf_resample_noalloc(int n_particles, size_t floats_per_particle, uint64_t seed,
                           uint32_t ensemble_id, uint64_t analysis_index, const double* logw,
                           const float* state_in, float* state_out, int32_t* parents,
                           void* stream);

/* Largest admissible scheme step of the current ensemble by eq. swecfl with Courant 0.8:
 * 0.8 * 1/4 * min(dx / max(|u| + c), dy / max(|v| + c)).  Waits for the stream.  Returns
 * IEWPF_E_CFL (and still writes *dt_out) when dt / n_sub exceeds it. */
int iewpf_check_cfl(iewpf_ctx* ctx, const float* state, double* dt_out, void* stream);

/* Copies a context constant or workspace to host for inspection (waits for the stream).
 * which: 0 xi [Ne][NR] f32, 1 nu~ [Ne][NR] f32, 2 r' [Ne][NR] f32, 3 S 2x2 f64,
 * 4 S_c 2x2 f64, 5 A^{1/2} 49x49 f64, 6 pull windows [2][3][W][W] f32 with W given by
 * iewpf_window_size, 7 S d of the last analysis [Ne][n_obs][2] f64, 8 model-error SOAR
 * stencil 5x5 f64, 9 the full S [2 n_obs][2 n_obs] f64 of the last full-covariance analysis,
 * 10 the parents [Ne] int32 of the last standard-particle-filter analysis (scheme 2).
 * bytes must equal the buffer size. */
int iewpf_read_buffer(iewpf_ctx* ctx, int which, void* host_out, size_t bytes, void* stream);

/* Window extents (x, y) of the stored pull windows (2r+1 or the folded grid size). */
int iewpf_window_size(iewpf_ctx* ctx, int32_t* wx, int32_t* wy);

/* Picks the stencil's rows-per-wave strip by timing candidate heights (16..96) on `state`
 * (read only; results go to the context's scratch buffer).  Waits for the stream; writes
 * the chosen height to *strip_out.  Later calls on ctx use it. */
int iewpf_autotune(iewpf_ctx* ctx, const float* state, int32_t* strip_out, void* stream);

/* Sets the stencil's rows-per-wave strip height directly (1 <= rows; heights above ny mean
 * one strip per column block).  Results do not depend on it.  Later calls on ctx use it;
 * batches created before keep the height they were built with.  IEWPF_E_ARG for rows < 1. */
int iewpf_set_strip_rows(iewpf_ctx* ctx, int rows);

/* ---- several ensembles of uneven grid and size in one captured cycle ------------------
 * A batch groups n contexts (same dt and n_sub) and their state buffers.  Each scheme step
 * launches every ensemble's own kernel (in the form its context chose) on up to eight side
 * streams forked from the cycle's stream and joined back, so a captured graph runs them as
 * parallel branches; with IEWPF_BATCH_SPLIT=0 in the environment at creation, one launch
 * over a device table of (grid, buffers, wave range) jobs covers all ensembles instead (the
 * strip form).  The model-error fields of all noisy model steps of a cycle are drawn ahead
 * per ensemble, and the analyses run per ensemble on the side streams.  Contexts and states
 * are owned by the caller and must outlive the batch.  n <= 16. */
typedef struct iewpf_batch iewpf_batch;
int iewpf_batch_create(iewpf_ctx* const* ctxs, float* const* states, int n, iewpf_batch** out);
void iewpf_batch_destroy(iewpf_batch* b);

/* Fixed observation cells of ensemble e (moorings; host [2*n_obs] of (j, k)): builds and
 * uploads its index lists once.  Waits for the stream. */
int iewpf_batch_set_cells(iewpf_batch* b, int e, const int32_t* cells_host, int n_obs,
                          void* stream);

/* One data-assimilation cycle of every ensemble: n_model_steps model steps (model error
 * after every step but the last, streams first_step + s), then one IEWPF analysis per
 * ensemble (stream analysis_index) with observation values y_host[e] (host float64
 * [n_obs_e][2] for the cells set above).  use_graph != 0: the first call captures the whole
 * cycle into one hipGraph (on an internal stream ordered after `stream`) and later calls
 * replay it; the cycle's first kernel copies the step and analysis indices and y from the
 * library's pinned, device-mapped buffers (written by the host before each replay) into
 * device memory, and its last kernel writes every ensemble's status words back there.  A
 * different n_model_steps recaptures.  The call waits for the cycle and returns the first
 * ensemble's analysis error as iewpf_assimilate does (IEWPF_E_BETA, IEWPF_E_NONFINITE; the
 * message names the ensemble; an ensemble whose analysis stopped before writing keeps its
 * forecast). */
int iewpf_batch_cycle(iewpf_batch* b, int n_model_steps, uint64_t first_step,
                      uint64_t analysis_index, const double* const* y_host, int use_graph,
                      void* stream);

/* ---- learned surrogate forecast ----------------------------------------------------------
 * A 6-layer convolutional network (3x3 kernels, periodic padding, 3 -> 48 -> 48 -> 48 -> 48
 * -> 48 -> 3, ReLU after the first five) that maps an ensemble state to the state one
 * forecast window (10 model steps) later: psi' = psi + s * net((psi - mu) / sigma), per
 * channel mu, sigma, s.  It runs in BF16 on the matrix cores with FP32 accumulation;
 * parameters are FP32 master weights trained with Adam by the library's own forward and
 * backward kernels.  The plain solver is its fallback: particles whose relative mass
 * drift exceeds a tolerance are re-stepped.  Parameter vector layout: for each layer
 * L = 0..5, weights [C_out][C_in][3][3] then biases [C_out] (float32). */
typedef struct iewpf_net iewpf_net;
/* Network with workspaces for up to max_cells = batch * ny * nx cells. */
int iewpf_net_create(int max_cells, iewpf_net** out);
void iewpf_net_destroy(iewpf_net* net);
size_t iewpf_net_num_params(const iewpf_net* net);
/* Copy host parameters in (resets the Adam state) / out; wait for the stream. */
int iewpf_net_set_params(iewpf_net* net, const float* host, size_t count, void* stream);
int iewpf_net_get_params(iewpf_net* net, float* host, size_t count, void* stream);
/* Normalisation statistics of training pairs x, target (device float32 [B][3][H][W] each),
 * per channel in float64: stats_out (host double [9]) = mu[3] (mean of x), sigma[3] (standard
 * deviation of x, n - 1 in the denominator, plus 1e-6), scale[3] (standard deviation of
 * target - x, plus 1e-9): the arguments of iewpf_net_set_norm.  Allocates and frees a small
 * device buffer; waits for the stream. */
int iewpf_norm_stats(const float* x, const float* target, int B, int H, int W, double* stats_out,
                     void* stream);
/* Per-channel normalisation mu, sigma (inputs) and output scale s (3 floats each, host). */
int iewpf_net_set_norm(iewpf_net* net, const float* mu, const float* sigma, const float* scale);
/* Number of model steps one application of the network stands in for (the forecast window
 * of its training pairs; 10 at creation).  The surrogate window and the surrogate drifter
 * forecast refuse other window lengths (IEWPF_E_ARG).  n_model_steps >= 1. */
int iewpf_net_set_horizon(iewpf_net* net, int n_model_steps);
/* state_out = state_in + s * net((state_in - mu) / sigma); device [B][3][H][W] float32 each
 * (state_out may equal state_in). */
int iewpf_net_forward(iewpf_net* net, const float* state_in, float* state_out, int B, int H,
                      int W, void* stream);
/* One Adam step (learning rate lr) on the MSE of net((x - mu)/sigma) against
 * (target - x)/s over all cells and channels; x, target device [B][3][H][W].  loss_out:
 * host pointer or NULL (when set the call waits and returns the loss before the update). */
int iewpf_net_train_step(iewpf_net* net, const float* x, const float* target, int B, int H, int W,
                         float lr, float* loss_out, void* stream);
/* Input of hidden layer `layer` (1..5) from the last forward or training call: BF16 bits
 * (round to nearest even of the ReLU output of layer `layer`-1), NHWC [cells][48], copied to
 * host uint16 [count]; count must equal 48 * cells of that call.  Waits for the stream.
 * For inspection and testing of the mixed-precision forward pass.  iewpf_net_forward runs
 * layers 0 and 1 as one fused pass and does not keep the input of layer 1; reading it after
 * such a forward returns IEWPF_E_ARG unless iewpf_net_keep_activations set the
 * layer-by-layer forward.  Training and gradient calls keep every layer. */
int iewpf_net_read_activation(iewpf_net* net, int layer, uint16_t* host, size_t count,
                              void* stream);
/* keep != 0: iewpf_net_forward runs layer by layer and writes every hidden activation to
 * device memory (for iewpf_net_read_activation); 0 (the default): layers 0 and 1 fused, so
 * layer 0's activation (1.44 GB of BF16 at 100 x 500x300 cells) stays on chip; the output is
 * bit-identical.  IEWPF_E_ARG for a NULL net. */
int iewpf_net_keep_activations(iewpf_net* net, int keep);
/* Loss gradient with respect to every parameter (host float [num_params]), without an
 * update; also the loss and the raw network output y (host float [B*H*W][3], NHWC, or
 * NULL).  Keeps every layer's pre-activation gradient for iewpf_net_read_gradient_signal
 * (five [cells][48] BF16 buffers, allocated when a call has more cells than any before).
 * Waits for the stream. */
int iewpf_net_gradients(iewpf_net* net, const float* x, const float* target, int B, int H, int W,
                        float* grads_host, float* loss_out, float* y_host, void* stream);
/* BF16 bits of the loss gradient with respect to the pre-activation of layer `layer`
 * (0..5; layer 5's is the rounded loss gradient of the output) from the last
 * iewpf_net_gradients call, NHWC [cells][C_out] with C_out 48 (layers 0..4) or 3 (layer 5),
 * copied to host uint16 [count]; count must equal C_out x the cells of that call.  Waits for
 * the stream.  For inspection and testing of the mixed-precision backward pass. */
int iewpf_net_read_gradient_signal(iewpf_net* net, int layer, uint16_t* host, size_t count,
                                   void* stream);
/* One surrogate forecast window of the ensemble in place: the network replaces
 * n_model_steps deterministic model steps (n_model_steps must equal the network's horizon,
 * IEWPF_E_ARG otherwise); every particle whose relative mass drift
 * |sum(H + eta') - sum(H + eta)| / sum(H + eta) exceeds drift_tol is re-stepped by the
 * plain solver from its saved state; then one model-error draw (stream first_step +
 * n_model_steps - 1) scaled by noise_scale is added to all particles.  n_fallback_out: host,
 * particles re-stepped; drift_out: host double [n_particles] or NULL.  Waits for the stream.
 * The network runs on as many particles at a time as its max_cells holds (at least one
 * particle's cells, else IEWPF_E_CAPACITY).  The first call allocates one state-sized
 * buffer in the context. */
int iewpf_surrogate_window(iewpf_ctx* ctx, iewpf_net* net, float* state, int n_model_steps,
                           uint64_t first_step, double drift_tol, double noise_scale,
                           int32_t* n_fallback_out, double* drift_out, void* stream);
/* The same window without host waits, so it can be captured in a graph or queued behind
 * other work: the flagged particles are re-stepped in place by plain scheme launches over
 * all particles in which the unflagged particles' workgroups return at once (the state
 * equals iewpf_surrogate_window's bit for bit).  n_fallback_dev: device int32, receives the
 * number of re-stepped particles; drift_dev: device double [n_particles] or NULL.  Does not
 * wait for the stream.  Its work buffers are those of iewpf_surrogate_window, allocated by
 * the first call of either form on the context: make that call outside a graph capture. */
int iewpf_surrogate_window_async(iewpf_ctx* ctx, iewpf_net* net, float* state, int n_model_steps,
                                 uint64_t first_step, double drift_tol, double noise_scale,
                                 int32_t* n_fallback_dev, double* drift_dev, void* stream);

/* Drifter forecast with the surrogate standing in for the model: n_windows windows of
 * steps_per_window model steps, each one iewpf_surrogate_window (plain re-step of the
 * particles whose mass drift exceeds drift_tol) followed by one model-error draw scaled by
 * noise_scale (stream first_step + (w + 1) steps_per_window - 1, tag 1).  Within a window the
 * drifters take steps_per_window Heun steps of dt in the states interpolated linearly in time
 * between the window's start and its (deterministic) end.  pos, traj as in
 * iewpf_forecast_drifters (traj: [n_windows steps_per_window + 1][...] or NULL);
 * n_fallback_out: host, re-stepped particles summed over the windows (or NULL).  Waits for
 * the stream.  Allocates one state-sized buffer in the context on its first call. */
int iewpf_forecast_drifters_surrogate(iewpf_ctx* ctx, iewpf_net* net, float* state, double* pos,
                                      int n_drifters, int n_windows, int steps_per_window,
                                      uint64_t first_step, double drift_tol, double noise_scale,
                                      double* traj, int32_t* n_fallback_out, void* stream);

/* Per-kernel timing with HIP events recorded around every launch on the call's stream
 * (for measurement; off by default).  iewpf_set_trace(ctx, 1) starts a fresh record;
 * iewpf_trace_read waits for the recorded events and returns, per kernel kind, the total
 * milliseconds and launch count since the last start.  Kinds: 0 scheme step (both RK
 * stages), 1 model-error normals, 2 SOAR, 3 geostrophic add (model error / initial state),
 * 4 innovations (full-covariance path), 5 innovations (other paths) + xi/nu draws + dot
 * products, 6 beta/alpha, 7 coarse posterior field, 8 analysis update pass, 9 scheme step
 * with the model error of its model step fused in.  n_kinds <= 16.  At most 8192 launches
 * are recorded; later launches are not timed. */
int iewpf_set_trace(iewpf_ctx* ctx, int on);
int iewpf_trace_read(iewpf_ctx* ctx, double* ms_out, int32_t* count_out, int n_kinds);

const char* iewpf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IEWPF_H */
