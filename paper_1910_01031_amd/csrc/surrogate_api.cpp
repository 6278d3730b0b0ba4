// extern "C" entry points of the learned surrogate (declared in include/iewpf.h): the
// network object (FP32 master weights, Adam moments, BF16 forward/transposed layouts,
// activation workspaces), its forward pass on ensembles, one training step, gradients
// for inspection, and the surrogate forecast window with the mass-drift guard and the
// plain-solver fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace {
constexpr int kLayers = 6;
constexpr int kCh[kLayers + 1] = {3, 48, 48, 48, 48, 48, 3};
constexpr int kChunkCells = 4096;  // cells per weight-gradient partial sum
int pad_to(int x, int m) { return (x + m - 1) / m * m; }
}  // namespace

struct iewpf_net {
  int max_cells = 0;
  long long last_cells = 0;  // cells of the last forward / training call
  size_t np = 0;
  size_t woff[kLayers], boff[kLayers];
  int Kf[kLayers], Npf[kLayers], Kd[kLayers], Npd[kLayers];
  float* p = nullptr;      // FP32 master parameters
  float* g = nullptr;      // gradients
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  int t = 0;
  uint16_t* wf[kLayers] = {};
  uint16_t* wd[kLayers] = {};
  uint16_t* act[kLayers] = {};  // act[i] = input of layer i (i >= 1), NHWC 48 channels
  float* y = nullptr;           // training output [cells][3]
  uint16_t* g5 = nullptr;       // loss gradient [cells][3]
  uint16_t* ga = nullptr;       // pre-activation gradients [cells][48] (ping-pong)
  uint16_t* gb = nullptr;
  float* wpart = nullptr;
  float* bpart = nullptr;
  float* lpart = nullptr;
  float* h_loss = nullptr;
  int loss_blocks = 256;
  float mu[3] = {0, 0, 0}, sig[3] = {1, 1, 1}, s[3] = {1, 1, 1};
  int horizon = 10;  // model steps one application of the network stands in for
  int keep_act = 0;  // forward layer by layer, every hidden activation to HBM (inspection)
  unsigned act_valid = 0;  // bit L: act[L] holds the last call's input of layer L
  // pre-activation gradients of layers 0..4 kept by iewpf_net_gradients ([cells][48] BF16
  // each, allocated on its first call for that call's cells); layer 5's is g5
  uint16_t* gkeep[kLayers - 1] = {};
  long long gkeep_cells = 0;
  long long gkeep_last = 0;  // cells of the last iewpf_net_gradients call
};

namespace iewpf {
namespace {

void free_net(iewpf_net* n) {
  if (!n) return;
  void* bufs[] = {n->p, n->g, n->m, n->v, n->y, n->g5, n->ga, n->gb, n->wpart, n->bpart, n->lpart};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int i = 0; i < kLayers - 1; ++i)
    if (n->gkeep[i]) (void)hipFree(n->gkeep[i]);
  for (int i = 0; i < kLayers; ++i) {
    if (n->wf[i]) (void)hipFree(n->wf[i]);
    if (n->wd[i]) (void)hipFree(n->wd[i]);
    if (n->act[i]) (void)hipFree(n->act[i]);
  }
  if (n->h_loss) (void)hipHostFree(n->h_loss);
  delete n;
}

ConvArgs conv_args(const iewpf_net* n, int layer, int B, int H, int W) {
  ConvArgs A{};
  A.B = B;
  A.H = H;
  A.W = W;
  A.cin = kCh[layer];
  A.cout = kCh[layer + 1];
  A.K = 9 * A.cin;
  A.Kpad = n->Kf[layer];
  A.Npad = n->Npf[layer];
  A.wt = n->wf[layer];
  A.bias = n->p + n->boff[layer];
  for (int c = 0; c < 3; ++c) {
    A.mu[c] = n->mu[c];
    A.isig[c] = 1.0f / n->sig[c];
    A.s[c] = n->s[c];
  }
  return A;
}

// Layers 0..4 of the forward pass (activations kept for the backward pass); layer 5 by the
// caller (residual into a state, or raw output for training).
void forward_hidden(iewpf_net* n, const float* state, int B, int H, int W, hipStream_t s) {
  n->last_cells = (long long)B * H * W;
  for (int L = 0; L < 5; ++L) {
    ConvArgs A = conv_args(n, L, B, H, W);
    A.in = L == 0 ? static_cast<const void*>(state) : static_cast<const void*>(n->act[L]);
    A.out = n->act[L + 1];
    launch_conv(A, L == 0 ? kInStateNorm : kInNhwcVec, kOutReluBf16, s);
  }
  n->act_valid = 0x3Eu;  // layers 1..5
}

// Inference forward with layers 0 and 1 fused (layer 0's activation stays on chip), then
// layers 2..5 one by one.  Returns false (nothing launched) when the first pair has no fused
// kernel.
bool forward_fused(iewpf_net* n, const float* state_in, float* state_out, int B, int H, int W,
                   hipStream_t s) {
  ConvArgs L0 = conv_args(n, 0, B, H, W), L1 = conv_args(n, 1, B, H, W);
  L0.in = state_in;
  L1.out = n->act[2];
  if (!launch_conv_pair(L0, kInStateNorm, L1, kOutReluBf16, s)) return false;
  for (int L = 2; L < 5; ++L) {
    ConvArgs A = conv_args(n, L, B, H, W);
    A.in = n->act[L];
    A.out = n->act[L + 1];
    launch_conv(A, kInNhwcVec, kOutReluBf16, s);
  }
  ConvArgs L5 = conv_args(n, 5, B, H, W);
  L5.in = n->act[5];
  L5.out = state_out;
  L5.state_in = state_in;
  launch_conv(L5, kInNhwcVec, kOutResidState, s);
  n->last_cells = (long long)B * H * W;
  n->act_valid = 0x3Cu;  // layers 2..5
  return true;
}

void prep_all(iewpf_net* n, hipStream_t s) {
  for (int L = 0; L < kLayers; ++L)
    launch_prep_weights(n->p + n->woff[L], kCh[L], kCh[L + 1], n->Kf[L], n->Npf[L], n->Kd[L],
                        n->Npd[L], n->wf[L], L > 0 ? n->wd[L] : nullptr, s);
}

// Forward (training output), MSE and backward: fills n->g; loss partials in n->lpart.
// keep: the pre-activation gradient of layer L - 1 goes to keep[L - 1] instead of the
// ping-pong buffers (inspection).
void forward_backward(iewpf_net* n, const float* x, const float* tgt, int B, int H, int W,
                      hipStream_t s, uint16_t* const* keep = nullptr) {
  const int cells = B * H * W;
  forward_hidden(n, x, B, H, W, s);
  ConvArgs A5 = conv_args(n, 5, B, H, W);
  A5.in = n->act[5];
  A5.out = n->y;
  launch_conv(A5, kInNhwcVec, kOutF32, s);
  launch_mse(n->y, x, tgt, B, H, W, n->s, n->g5, n->lpart, n->loss_blocks, s);
  const int nchunks = (cells + kChunkCells - 1) / kChunkCells;
  const uint16_t* gz = n->g5;  // gradient w.r.t. the pre-activation of layer L
  int gch = 3;
  uint16_t* bufs[2] = {n->ga, n->gb};
  for (int L = 5; L >= 0; --L) {
    ConvArgs A = conv_args(n, L, B, H, W);
    A.in = L == 0 ? static_cast<const void*>(x) : static_cast<const void*>(n->act[L]);
    launch_wgrad(A, L == 0 ? kInStateNorm : kInNhwcVec, gz, gch, kChunkCells, n->wpart, s);
    launch_bgrad(gz, gch, cells, kChunkCells, n->bpart, s);
    launch_reduce_grads(n->wpart, n->bpart, nchunks, kCh[L], kCh[L + 1], n->Kf[L], n->Npf[L],
                        n->g + n->woff[L], n->g + n->boff[L], s);
    if (L == 0) break;
    // input gradient of layer L, masked by the ReLU of layer L-1 (its output = act[L])
    ConvArgs D{};
    D.B = B;
    D.H = H;
    D.W = W;
    D.cin = kCh[L + 1];
    D.cout = kCh[L];
    D.K = 9 * D.cin;
    D.Kpad = n->Kd[L];
    D.Npad = n->Npd[L];
    D.wt = n->wd[L];
    D.bias = nullptr;
    D.in = gz;
    D.mask = n->act[L];
    uint16_t* out = keep ? keep[L - 1] : bufs[L & 1];
    D.out = out;
    launch_conv(D, gch % 8 == 0 ? kInNhwcVec : kInNhwcSmall, kOutMaskBf16, s);
    gz = out;
    gch = kCh[L];
  }
}

}  // namespace

int net_max_cells(const iewpf_net* n) { return n ? n->max_cells : 0; }
int net_horizon(const iewpf_net* n) { return n ? n->horizon : 0; }

}  // namespace iewpf

using namespace iewpf;

extern "C" {

int iewpf_net_create(int max_cells, iewpf_net** out) {
  if (!out || max_cells <= 0) return fail(IEWPF_E_ARG, "invalid argument");
  *out = nullptr;
  iewpf_net* n = new iewpf_net();
  n->max_cells = max_cells;
  size_t off = 0;
  for (int L = 0; L < kLayers; ++L) {
    n->woff[L] = off;
    off += (size_t)kCh[L + 1] * kCh[L] * 9;
    n->boff[L] = off;
    off += kCh[L + 1];
    n->Kf[L] = pad_to(9 * kCh[L], 32);
    n->Npf[L] = pad_to(kCh[L + 1], 16);
    n->Kd[L] = pad_to(9 * kCh[L + 1], 32);
    n->Npd[L] = pad_to(kCh[L], 16);
  }
  n->np = off;
  const int nchunks = (max_cells + kChunkCells - 1) / kChunkCells;
  bool ok = hipMalloc(reinterpret_cast<void**>(&n->p), n->np * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->g), n->np * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->m), n->np * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->v), n->np * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->y), (size_t)max_cells * 3 * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->g5), (size_t)max_cells * 3 * 2) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->ga), (size_t)max_cells * 48 * 2) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->gb), (size_t)max_cells * 48 * 2) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->wpart), (size_t)nchunks * 48 * 448 * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->bpart), (size_t)nchunks * 48 * 4) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&n->lpart), (size_t)n->loss_blocks * 4) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&n->h_loss), (size_t)n->loss_blocks * 4) == hipSuccess;
  for (int L = 0; ok && L < kLayers; ++L) {
    ok = hipMalloc(reinterpret_cast<void**>(&n->wf[L]), (size_t)n->Npf[L] * n->Kf[L] * 2) == hipSuccess;
    if (ok && L > 0)
      ok = hipMalloc(reinterpret_cast<void**>(&n->wd[L]), (size_t)n->Npd[L] * n->Kd[L] * 2) == hipSuccess;
    if (ok && L > 0)
      ok = hipMalloc(reinterpret_cast<void**>(&n->act[L]), (size_t)max_cells * 48 * 2) == hipSuccess;
  }
  if (!ok) {
    free_net(n);
    return fail(IEWPF_E_HIP, "network allocation failed");
  }
  (void)hipMemset(n->p, 0, n->np * 4);
  (void)hipMemset(n->m, 0, n->np * 4);
  (void)hipMemset(n->v, 0, n->np * 4);
  prep_all(n, nullptr);
  if (hipDeviceSynchronize() != hipSuccess) {
    free_net(n);
    return fail(IEWPF_E_HIP, "network initialisation failed");
  }
  *out = n;
  return 0;
}

void iewpf_net_destroy(iewpf_net* n) {
  if (!n) return;
  (void)hipDeviceSynchronize();
  free_net(n);
}

size_t iewpf_net_num_params(const iewpf_net* n) { return n ? n->np : 0; }

int iewpf_net_set_params(iewpf_net* n, const float* host, size_t count, void* stream) {
  if (!n || !host || count != n->np) return fail(IEWPF_E_ARG, "parameter count mismatch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  IEWPF_HIP_TRY(hipMemcpy(n->p, host, n->np * 4, hipMemcpyHostToDevice));
  IEWPF_HIP_TRY(hipMemset(n->m, 0, n->np * 4));
  IEWPF_HIP_TRY(hipMemset(n->v, 0, n->np * 4));
  n->t = 0;
  prep_all(n, s);
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int iewpf_net_get_params(iewpf_net* n, float* host, size_t count, void* stream) {
  if (!n || !host || count != n->np) return fail(IEWPF_E_ARG, "parameter count mismatch");
  IEWPF_HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  IEWPF_HIP_TRY(hipMemcpy(host, n->p, n->np * 4, hipMemcpyDeviceToHost));
  return 0;
}

int iewpf_net_set_norm(iewpf_net* n, const float* mu, const float* sigma, const float* scale) {
  if (!n || !mu || !sigma || !scale) return fail(IEWPF_E_ARG, "NULL argument");
  for (int c = 0; c < 3; ++c) {
    if (!(sigma[c] > 0) || !(scale[c] > 0)) return fail(IEWPF_E_ARG, "sigma and scale must be > 0");
    n->mu[c] = mu[c];
    n->sig[c] = sigma[c];
    n->s[c] = scale[c];
  }
  return 0;
}

int iewpf_norm_stats(const float* x, const float* target, int B, int H, int W, double* stats_out,
                     void* stream) {
  if (!x || !target || !stats_out || B < 1 || H < 1 || W < 1 || (long long)B * H * W < 2)
    return fail(IEWPF_E_ARG, "invalid argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* buf = nullptr;
  IEWPF_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&buf), sizeof(double) * (channel_stats_parts() + 9)));
  launch_channel_stats(x, target, B, H * W, buf, buf + channel_stats_parts(), s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(stats_out, buf + channel_stats_parts(), sizeof(double) * 9,
                                          hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(IEWPF_E_HIP, std::string("normalisation statistics: ") + hipGetErrorString(e));
  return 0;
}

int iewpf_net_set_horizon(iewpf_net* n, int n_model_steps) {
  if (!n || n_model_steps < 1) return fail(IEWPF_E_ARG, "the horizon must be at least one model step");
  n->horizon = n_model_steps;
  return 0;
}

int iewpf_net_forward(iewpf_net* n, const float* state_in, float* state_out, int B, int H, int W,
                      void* stream) {
  if (!n || !state_in || !state_out || B <= 0 || H < 1 || W < 1) return fail(IEWPF_E_ARG, "invalid argument");
  if ((long long)B * H * W > n->max_cells) return fail(IEWPF_E_CAPACITY, "more cells than max_cells");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (n->keep_act || !forward_fused(n, state_in, state_out, B, H, W, s)) {
    forward_hidden(n, state_in, B, H, W, s);
    ConvArgs A5 = conv_args(n, 5, B, H, W);
    A5.in = n->act[5];
    A5.out = state_out;
    A5.state_in = state_in;
    launch_conv(A5, kInNhwcVec, kOutResidState, s);
  }
  IEWPF_HIP_TRY(hipGetLastError());
  return 0;
}

int iewpf_net_keep_activations(iewpf_net* n, int keep) {
  if (!n) return fail(IEWPF_E_ARG, "invalid argument");
  n->keep_act = keep != 0;
  return 0;
}

int iewpf_net_train_step(iewpf_net* n, const float* x, const float* target, int B, int H, int W,
                         float lr, float* loss_out, void* stream) {
  if (!n || !x || !target || B <= 0 || !(lr > 0)) return fail(IEWPF_E_ARG, "invalid argument");
  if ((long long)B * H * W > n->max_cells) return fail(IEWPF_E_CAPACITY, "more cells than max_cells");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  forward_backward(n, x, target, B, H, W, s);
  n->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)n->t), c2 = 1.0f - std::pow(b2, (float)n->t);
  launch_adam(n->p, n->g, n->m, n->v, (int)n->np, lr, b1, b2, 1e-8f, c1, c2, s);
  prep_all(n, s);
  IEWPF_HIP_TRY(hipGetLastError());
  if (loss_out) {
    IEWPF_HIP_TRY(hipMemcpyAsync(n->h_loss, n->lpart, n->loss_blocks * 4, hipMemcpyDeviceToHost, s));
    IEWPF_HIP_TRY(hipStreamSynchronize(s));
    double acc = 0.0;
    for (int i = 0; i < n->loss_blocks; ++i) acc += n->h_loss[i];
    *loss_out = (float)acc;
  }
  return 0;
}

int iewpf_net_read_activation(iewpf_net* n, int layer, uint16_t* host, size_t count, void* stream) {
  if (!n || !host || layer < 1 || layer > 5) return fail(IEWPF_E_ARG, "invalid argument");
  if (count != (size_t)48 * n->last_cells || n->last_cells == 0)
    return fail(IEWPF_E_ARG, "count must be 48 x the cells of the last call");
  if (!(n->act_valid >> layer & 1u))
    return fail(IEWPF_E_ARG, "the last forward kept no input of layer " + std::to_string(layer) +
                                 " (fused layer pairs); call iewpf_net_keep_activations first");
  IEWPF_HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  IEWPF_HIP_TRY(hipMemcpy(host, n->act[layer], count * 2, hipMemcpyDeviceToHost));
  return 0;
}

int iewpf_net_read_gradient_signal(iewpf_net* n, int layer, uint16_t* host, size_t count,
                                   void* stream) {
  if (!n || !host || layer < 0 || layer > 5) return fail(IEWPF_E_ARG, "invalid argument");
  const size_t ch = layer == 5 ? 3 : 48;
  if (n->gkeep_last == 0 || count != ch * (size_t)n->gkeep_last)
    return fail(IEWPF_E_ARG, "count must be C_out x the cells of the last iewpf_net_gradients call");
  IEWPF_HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  const uint16_t* src = layer == 5 ? n->g5 : n->gkeep[layer];
  IEWPF_HIP_TRY(hipMemcpy(host, src, count * 2, hipMemcpyDeviceToHost));
  return 0;
}

int iewpf_net_gradients(iewpf_net* n, const float* x, const float* target, int B, int H, int W,
                        float* grads_host, float* loss_out, float* y_host, void* stream) {
  if (!n || !x || !target || !grads_host) return fail(IEWPF_E_ARG, "invalid argument");
  if ((long long)B * H * W > n->max_cells) return fail(IEWPF_E_CAPACITY, "more cells than max_cells");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long cells = (long long)B * H * W;
  if (cells > n->gkeep_cells) {
    IEWPF_HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < kLayers - 1; ++i) {
      if (n->gkeep[i]) IEWPF_HIP_TRY(hipFree(n->gkeep[i]));
      n->gkeep[i] = nullptr;
    }
    n->gkeep_cells = 0;
    for (int i = 0; i < kLayers - 1; ++i)
      IEWPF_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&n->gkeep[i]), (size_t)cells * 48 * 2));
    n->gkeep_cells = cells;
  }
  forward_backward(n, x, target, B, H, W, s, n->gkeep);
  n->gkeep_last = cells;
  IEWPF_HIP_TRY(hipGetLastError());
  IEWPF_HIP_TRY(hipStreamSynchronize(s));
  IEWPF_HIP_TRY(hipMemcpy(grads_host, n->g, n->np * 4, hipMemcpyDeviceToHost));
  if (y_host) IEWPF_HIP_TRY(hipMemcpy(y_host, n->y, (size_t)B * H * W * 3 * 4, hipMemcpyDeviceToHost));
  if (loss_out) {
    IEWPF_HIP_TRY(hipMemcpy(n->h_loss, n->lpart, n->loss_blocks * 4, hipMemcpyDeviceToHost));
    double acc = 0.0;
    for (int i = 0; i < n->loss_blocks; ++i) acc += n->h_loss[i];
    *loss_out = (float)acc;
  }
  return 0;
}

}  // extern "C"
