"""ctypes binding of libiewpf.so (include/iewpf.h): argument marshalling only.

Device buffers are passed as torch tensors (their data pointers) and the HIP stream as
torch's current stream; every step of the forecast and analysis runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiewpf.so")

IEWPF_OK = 0
IEWPF_E_ARG = -1
IEWPF_E_SHAPE = -2
IEWPF_E_CFL = -3
IEWPF_E_NONFINITE = -4
IEWPF_E_BETA = -5
IEWPF_E_HIP = -6
IEWPF_E_CAPACITY = -7

EXPORTED = ("iewpf_create", "iewpf_destroy", "iewpf_init_ensemble", "iewpf_step_ensemble",
            "iewpf_perturb", "iewpf_assimilate", "iewpf_particle_scalars",
            "iewpf_observe_moorings", "iewpf_forecast_drifters", "iewpf_advect_drifters",
            "iewpf_resample", "iewpf_check_cfl", "iewpf_read_buffer", "iewpf_window_size",
            "iewpf_set_trace", "iewpf_trace_read", "iewpf_autotune", "iewpf_set_strip_rows",
            "iewpf_batch_create",
            "iewpf_batch_destroy", "iewpf_batch_set_cells", "iewpf_batch_cycle",
            "iewpf_net_create", "iewpf_net_destroy", "iewpf_net_num_params",
            "iewpf_net_set_params", "iewpf_net_get_params", "iewpf_net_set_norm",
            "iewpf_net_forward", "iewpf_net_train_step", "iewpf_net_read_activation",
            "iewpf_net_keep_activations",
            "iewpf_net_gradients",
            "iewpf_surrogate_window", "iewpf_surrogate_window_async",
            "iewpf_forecast_drifters_surrogate",
            "iewpf_set_full_innovation", "iewpf_set_scheme", "iewpf_last_error",
            "iewpf_observe_drifters", "iewpf_sir_log_weights", "iewpf_net_set_horizon",
            "iewpf_resample_noalloc", "iewpf_net_read_gradient_signal", "iewpf_norm_stats")

TRACE_KINDS = ("scheme_step", "me_normals", "soar", "gb_add", "innovation", "rand_dots",
               "beta_alpha", "posterior_coarse", "analysis_update", "scheme_step_noise",
               "soar_model_error")


class IewpfConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("H", ctypes.c_double),
                ("g", ctypes.c_double), ("f", ctypes.c_double), ("dt", ctypes.c_double),
                ("n_sub", ctypes.c_int32), ("theta", ctypes.c_double),
                ("c_omega", ctypes.c_int32), ("me_std", ctypes.c_double),
                ("me_L0", ctypes.c_double), ("init_std", ctypes.c_double),
                ("init_L0", ctypes.c_double), ("obs_sigma", ctypes.c_double),
                ("n_particles", ctypes.c_int32), ("max_obs", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("ensemble_id", ctypes.c_uint32)]


class IewpfObs(ctypes.Structure):
    _fields_ = [("j", ctypes.c_int32), ("k", ctypes.c_int32),
                ("y_hu", ctypes.c_double), ("y_hv", ctypes.c_double)]


class IewpfStats(ctypes.Structure):
    _fields_ = [("cbar", ctypes.c_double), ("beta", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("cstar_max", ctypes.c_double), ("c_min", ctypes.c_double),
                ("c_max", ctypes.c_double), ("argmin_beta", ctypes.c_int32),
                ("n_obs", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it is missing).  IEWPF_LIBRARY, when set, names another
    build of it (a tuning variant) in place of the in-tree one."""
    global _lib
    if _lib is not None:
        return _lib
    if path == LIB_PATH and os.environ.get("IEWPF_LIBRARY"):
        path = os.environ["IEWPF_LIBRARY"]
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1910_01031_amd/build.py "
                           "(the HIP library is required; there is no fallback)")
    # torch ships its own HIP runtime: load it first so that the library binds to the same
    # one (a second runtime loaded before torch's leaves torch without devices).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, u64, f64p = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
    lib.iewpf_create.argtypes = [ctypes.POINTER(IewpfConfig), ctypes.POINTER(vp)]
    lib.iewpf_destroy.argtypes = [vp]
    lib.iewpf_destroy.restype = None
    lib.iewpf_init_ensemble.argtypes = [vp, vp, vp, u64, vp]
    lib.iewpf_step_ensemble.argtypes = [vp, vp, i32, u64, i32, vp]
    lib.iewpf_perturb.argtypes = [vp, vp, u64, vp]
    lib.iewpf_assimilate.argtypes = [vp, vp, ctypes.POINTER(IewpfObs), i32, u64,
                                     ctypes.POINTER(IewpfStats), vp]
    lib.iewpf_particle_scalars.argtypes = [vp, f64p, vp]
    lib.iewpf_observe_moorings.argtypes = [vp, vp, vp, i32, u64, ctypes.POINTER(IewpfObs), vp]
    lib.iewpf_forecast_drifters.argtypes = [vp, vp, vp, i32, i32, u64, vp, vp]
    lib.iewpf_advect_drifters.argtypes = [vp, vp, vp, vp, i32, vp]
    lib.iewpf_resample.argtypes = [vp, vp, vp, u64, vp, vp]
    lib.iewpf_check_cfl.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.iewpf_read_buffer.argtypes = [vp, i32, vp, ctypes.c_size_t, vp]
    lib.iewpf_window_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.iewpf_autotune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.iewpf_set_strip_rows.argtypes = [vp, i32]
    lib.iewpf_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), i32,
                                       ctypes.POINTER(vp)]
    lib.iewpf_batch_destroy.argtypes = [vp]
    lib.iewpf_batch_destroy.restype = None
    lib.iewpf_batch_set_cells.argtypes = [vp, i32, vp, i32, vp]
    lib.iewpf_batch_cycle.argtypes = [vp, i32, u64, u64, ctypes.POINTER(vp), i32, vp]
    lib.iewpf_net_create.argtypes = [i32, ctypes.POINTER(vp)]
    lib.iewpf_net_destroy.argtypes = [vp]
    lib.iewpf_net_destroy.restype = None
    lib.iewpf_net_num_params.argtypes = [vp]
    lib.iewpf_net_set_params.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.iewpf_net_get_params.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.iewpf_net_set_norm.argtypes = [vp, vp, vp, vp]
    lib.iewpf_net_forward.argtypes = [vp, vp, vp, i32, i32, i32, vp]
    lib.iewpf_net_train_step.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_float), vp]
    lib.iewpf_net_read_activation.argtypes = [vp, i32, vp, ctypes.c_size_t, vp]
    lib.iewpf_net_keep_activations.argtypes = [vp, i32]
    lib.iewpf_net_gradients.argtypes = [vp, vp, vp, i32, i32, i32, vp,
                                        ctypes.POINTER(ctypes.c_float), vp, vp]
    lib.iewpf_surrogate_window.argtypes = [vp, vp, vp, i32, u64, ctypes.c_double,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                           vp, vp]
    lib.iewpf_surrogate_window_async.argtypes = [vp, vp, vp, i32, u64, ctypes.c_double,
                                                 ctypes.c_double, vp, vp, vp]
    lib.iewpf_forecast_drifters_surrogate.argtypes = [vp, vp, vp, vp, i32, i32, i32, u64,
                                                      ctypes.c_double, ctypes.c_double, vp,
                                                      ctypes.POINTER(ctypes.c_int32), vp]
    lib.iewpf_set_full_innovation.argtypes = [vp, i32]
    lib.iewpf_set_scheme.argtypes = [vp, i32]
    lib.iewpf_observe_drifters.argtypes = [vp, vp, vp, i32, ctypes.c_double, u64,
                                           ctypes.POINTER(IewpfObs), vp]
    lib.iewpf_sir_log_weights.argtypes = [vp, vp, ctypes.POINTER(IewpfObs), i32, ctypes.c_double,
                                          vp, vp, vp]
    lib.iewpf_net_set_horizon.argtypes = [vp, i32]
    lib.iewpf_net_read_gradient_signal.argtypes = [vp, i32, vp, ctypes.c_size_t, vp]
    lib.iewpf_norm_stats.argtypes = [vp, vp, i32, i32, i32, f64p, vp]
    lib.iewpf_resample_noalloc.argtypes = [i32, ctypes.c_size_t, u64, ctypes.c_uint32, u64, vp, vp,
                                           vp, vp, vp]
    lib.iewpf_set_trace.argtypes = [vp, i32]
    lib.iewpf_trace_read.argtypes = [vp, f64p, vp, i32]
    lib.iewpf_net_num_params.restype = ctypes.c_size_t
    lib.iewpf_last_error.restype = ctypes.c_char_p
    lib.iewpf_last_error.argtypes = []
    for name in EXPORTED:
        if name not in ("iewpf_destroy", "iewpf_last_error", "iewpf_batch_destroy",
                        "iewpf_net_destroy", "iewpf_net_num_params"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class IewpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"iewpf error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != 0:
        raise IewpfError(rc, load().iewpf_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_config(cfg, max_obs: int = 256) -> IewpfConfig:
    """iewpf_config from a workloads.Config-like object."""
    return IewpfConfig(nx=cfg.nx, ny=cfg.ny, dx=cfg.dx, dy=cfg.dy, H=cfg.H, g=cfg.g, f=cfg.f,
                       dt=cfg.dt, n_sub=cfg.n_sub, theta=cfg.theta, c_omega=cfg.c_omega,
                       me_std=cfg.me_std, me_L0=cfg.L0, init_std=cfg.init_std,
                       init_L0=cfg.init_L, obs_sigma=cfg.obs_sigma,
                       n_particles=cfg.n_particles, max_obs=max_obs, seed=cfg.seed,
                       ensemble_id=cfg.ensemble_id)


def obs_array(cells: np.ndarray, y: np.ndarray):
    n = len(cells)
    arr = (IewpfObs * max(n, 1))()
    for o in range(n):
        arr[o].j = int(cells[o, 0])
        arr[o].k = int(cells[o, 1])
        arr[o].y_hu = float(y[o, 0])
        arr[o].y_hv = float(y[o, 1])
    return arr


class Context:
    """Owns one iewpf_ctx; methods mirror the C entry points."""

    def __init__(self, cfg, max_obs: int = 256):
        lib = load()
        self.cfg = cfg
        self.max_obs = max_obs
        self._c = make_config(cfg, max_obs)
        h = ctypes.c_void_p()
        _check(lib.iewpf_create(ctypes.byref(self._c), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().iewpf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_ensemble(self, state, base=None, stream_index: int = 0, stream=None):
        _check(load().iewpf_init_ensemble(self.h, _ptr(state), _ptr(base), stream_index,
                                          _stream(stream)))

    def step_ensemble(self, state, n_model_steps: int, first_step: int = 0,
                      noise_on_last: bool = True, stream=None):
        _check(load().iewpf_step_ensemble(self.h, _ptr(state), n_model_steps, first_step,
                                          int(noise_on_last), _stream(stream)))

    def perturb(self, state, step_index: int, stream=None):
        _check(load().iewpf_perturb(self.h, _ptr(state), step_index, _stream(stream)))

    def assimilate(self, state, cells: np.ndarray, y: np.ndarray, analysis_index: int,
                   want_stats: bool = True, stream=None, obs=None):
        if obs is None:
            obs = obs_array(cells, y)
        n = len(cells) if cells is not None else len(obs)
        st = IewpfStats()
        _check(load().iewpf_assimilate(self.h, _ptr(state), obs, n, analysis_index,
                                       ctypes.byref(st) if want_stats else None,
                                       _stream(stream)))
        return st.as_dict() if want_stats else None

    def set_scheme(self, scheme):
        """0 / False: two-stage IEWPF (default); 1 / True: the one-stage scheme; 2: the
        standard particle filter (SIR weights and residual resampling)."""
        _check(load().iewpf_set_scheme(self.h, int(scheme)))

    def sir_parents(self) -> np.ndarray:
        """Parents of the last standard-particle-filter analysis (buffer 10)."""
        return self.read_buffer(10, (self.cfg.n_particles,), np.int32)

    def set_full_innovation(self, on: bool):
        _check(load().iewpf_set_full_innovation(self.h, 1 if on else 0))

    def particle_scalars(self, stream=None) -> np.ndarray:
        out = np.zeros((self.cfg.n_particles, 8))
        _check(load().iewpf_particle_scalars(self.h, out.ctypes.data, _stream(stream)))
        return out

    def observe_moorings(self, truth, cells: np.ndarray, analysis_index: int, stream=None):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        n = len(cells)
        arr = (IewpfObs * max(n, 1))()
        _check(load().iewpf_observe_moorings(self.h, _ptr(truth), cells.ctypes.data, n,
                                             analysis_index, arr, _stream(stream)))
        return np.array([[arr[o].y_hu, arr[o].y_hv] for o in range(n)])

    def observe_drifters(self, pos_now, pos_prev, dt_obs: float, analysis_index: int,
                         stream=None):
        """Drifter observations (device float64 [n][2] positions): returns (cells int32
        [n][2], y float64 [n][2])."""
        n = int(pos_now.shape[0])
        arr = (IewpfObs * max(n, 1))()
        _check(load().iewpf_observe_drifters(self.h, _ptr(pos_now), _ptr(pos_prev), n, dt_obs,
                                             analysis_index, arr, _stream(stream)))
        cells = np.array([[arr[o].j, arr[o].k] for o in range(n)], dtype=np.int32).reshape(n, 2)
        y = np.array([[arr[o].y_hu, arr[o].y_hv] for o in range(n)]).reshape(n, 2)
        return cells, y

    def sir_log_weights(self, state, cells: np.ndarray, y: np.ndarray, logw, w=None,
                        r_scale: float = 1.0, stream=None):
        """Standard-particle-filter log-weights into logw (device float64 [Ne]) and, when
        given, the normalised weights into w."""
        n = len(cells)
        _check(load().iewpf_sir_log_weights(self.h, _ptr(state), obs_array(cells, y), n,
                                            float(r_scale), _ptr(logw), _ptr(w), _stream(stream)))

    def forecast_drifters(self, state, pos, n_model_steps: int, first_step: int, traj=None,
                          stream=None):
        nd = pos.shape[1]
        _check(load().iewpf_forecast_drifters(self.h, _ptr(state), _ptr(pos), nd, n_model_steps,
                                              first_step, _ptr(traj), _stream(stream)))

    def advect_drifters(self, psi_n, psi_np1, pos, stream=None):
        _check(load().iewpf_advect_drifters(self.h, _ptr(psi_n), _ptr(psi_np1), _ptr(pos),
                                            pos.shape[1], _stream(stream)))

    def resample(self, state, logw, analysis_index: int, parents, stream=None):
        _check(load().iewpf_resample(self.h, _ptr(state), _ptr(logw), analysis_index,
                                     _ptr(parents), _stream(stream)))

    def check_cfl(self, state, stream=None):
        """Returns (dt_cfl, ok)."""
        dt = ctypes.c_double()
        rc = load().iewpf_check_cfl(self.h, _ptr(state), ctypes.byref(dt), _stream(stream))
        if rc not in (0, IEWPF_E_CFL):
            _check(rc)
        return dt.value, rc == 0

    def autotune(self, state, stream=None) -> int:
        out = ctypes.c_int32()
        _check(load().iewpf_autotune(self.h, _ptr(state), ctypes.byref(out), _stream(stream)))
        return out.value

    def set_strip_rows(self, rows: int):
        _check(load().iewpf_set_strip_rows(self.h, int(rows)))

    def set_trace(self, on: bool):
        _check(load().iewpf_set_trace(self.h, int(on)))

    def trace_read(self):
        """{kind: (total_ms, launches)} since the last set_trace(True)."""
        n = len(TRACE_KINDS)
        ms = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int32)
        _check(load().iewpf_trace_read(self.h, ms.ctypes.data, cnt.ctypes.data, n))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(TRACE_KINDS)}

    def window_size(self):
        wx, wy = ctypes.c_int32(), ctypes.c_int32()
        _check(load().iewpf_window_size(self.h, ctypes.byref(wx), ctypes.byref(wy)))
        return wx.value, wy.value

    def read_buffer(self, which: int, shape, dtype, stream=None) -> np.ndarray:
        out = np.zeros(shape, dtype=dtype)
        _check(load().iewpf_read_buffer(self.h, which, out.ctypes.data, out.nbytes,
                                        _stream(stream)))
        return out


class Batch:
    """Several contexts stepped by one launch per scheme step (iewpf_batch_*)."""

    def __init__(self, contexts, states):
        lib = load()
        n = len(contexts)
        self.contexts = list(contexts)
        self.states = list(states)
        hs = (ctypes.c_void_p * n)(*[c.h.value for c in contexts])
        ps = (ctypes.c_void_p * n)(*[t.data_ptr() for t in states])
        h = ctypes.c_void_p()
        _check(lib.iewpf_batch_create(hs, ps, n, ctypes.byref(h)))
        self.h = h
        self.n_obs = [0] * n

    def close(self):
        if getattr(self, "h", None):
            load().iewpf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_cells(self, e: int, cells: np.ndarray, stream=None):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        _check(load().iewpf_batch_set_cells(self.h, e, cells.ctypes.data, len(cells), _stream(stream)))
        self.n_obs[e] = len(cells)

    def cycle(self, n_model_steps: int, first_step: int, analysis_index: int, y_list,
              use_graph: bool = False, stream=None):
        ys = [np.ascontiguousarray(y, dtype=np.float64) for y in y_list]
        self._keep = ys
        arr = (ctypes.c_void_p * len(ys))(*[y.ctypes.data for y in ys])
        _check(load().iewpf_batch_cycle(self.h, n_model_steps, first_step, analysis_index, arr,
                                        int(use_graph), _stream(stream)))


class Net:
    """The learned surrogate network (iewpf_net_*)."""

    def __init__(self, max_cells: int):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.iewpf_net_create(int(max_cells), ctypes.byref(h)))
        self.h = h
        self.num_params = int(lib.iewpf_net_num_params(h))

    def close(self):
        if getattr(self, "h", None):
            load().iewpf_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat: np.ndarray, stream=None):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(load().iewpf_net_set_params(self.h, flat.ctypes.data, flat.size, _stream(stream)))

    def get_params(self, stream=None) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        _check(load().iewpf_net_get_params(self.h, out.ctypes.data, out.size, _stream(stream)))
        return out

    def set_horizon(self, n_model_steps: int):
        """Model steps one application of the network stands in for (10 at creation)."""
        _check(load().iewpf_net_set_horizon(self.h, int(n_model_steps)))

    def set_norm(self, mu, sigma, scale):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (mu, sigma, scale)]
        self._norm = arrs
        _check(load().iewpf_net_set_norm(self.h, *[a.ctypes.data for a in arrs]))

    def forward(self, state_in, state_out, stream=None):
        B, _, H, W = state_in.shape
        _check(load().iewpf_net_forward(self.h, _ptr(state_in), _ptr(state_out), B, H, W,
                                        _stream(stream)))

    def train_step(self, x, target, lr: float, want_loss: bool = False, stream=None):
        B, _, H, W = x.shape
        loss = ctypes.c_float()
        _check(load().iewpf_net_train_step(self.h, _ptr(x), _ptr(target), B, H, W, lr,
                                           ctypes.byref(loss) if want_loss else None,
                                           _stream(stream)))
        return loss.value if want_loss else None

    def keep_activations(self, keep: bool = True) -> None:
        """Forward layer by layer, keeping every hidden activation (default: fused pairs)."""
        _check(load().iewpf_net_keep_activations(self.h, 1 if keep else 0))

    def read_activation(self, layer: int, cells: int, stream=None) -> np.ndarray:
        """BF16 bits (uint16 [cells][48]) of the input of hidden layer `layer` (1..5)."""
        out = np.zeros((cells, 48), dtype=np.uint16)
        _check(load().iewpf_net_read_activation(self.h, layer, out.ctypes.data, out.size,
                                                _stream(stream)))
        return out

    def read_gradient_signal(self, layer: int, cells: int, stream=None) -> np.ndarray:
        """BF16 bits (uint16 [cells][C_out]) of the pre-activation gradient of layer `layer`
        (0..5) from the last gradients call."""
        out = np.zeros((cells, 3 if layer == 5 else 48), dtype=np.uint16)
        _check(load().iewpf_net_read_gradient_signal(self.h, layer, out.ctypes.data, out.size,
                                                     _stream(stream)))
        return out

    def gradients(self, x, target, stream=None):
        """(grads float32 [num_params], loss, y float32 [B*H*W, 3])."""
        B, _, H, W = x.shape
        g = np.zeros(self.num_params, dtype=np.float32)
        y = np.zeros((B * H * W, 3), dtype=np.float32)
        loss = ctypes.c_float()
        _check(load().iewpf_net_gradients(self.h, _ptr(x), _ptr(target), B, H, W, g.ctypes.data,
                                          ctypes.byref(loss), y.ctypes.data, _stream(stream)))
        return g, loss.value, y


def norm_stats(x, target, stream=None):
    """Per-channel (mu, sigma, scale) of training pairs (device float32 [B][3][H][W])."""
    B, _, H, W = x.shape
    out = np.zeros(9)
    _check(load().iewpf_norm_stats(_ptr(x), _ptr(target), B, H, W, out.ctypes.data,
                                   _stream(stream)))
    return out[0:3].copy(), out[3:6].copy(), out[6:9].copy()


def resample_noalloc(logw, state_in, state_out, parents, seed: int, ensemble_id: int,
                     analysis_index: int, stream=None):
    """Residual resampling without allocation (iewpf_resample_noalloc): out of place."""
    n = int(state_in.shape[0])
    per = int(state_in[0].numel())
    _check(load().iewpf_resample_noalloc(n, per, seed, ensemble_id, analysis_index, _ptr(logw),
                                         _ptr(state_in), _ptr(state_out), _ptr(parents),
                                         _stream(stream)))


def surrogate_window(ctx, net, state, n_model_steps: int, first_step: int, drift_tol: float,
                     noise_scale: float, stream=None):
    """Returns (n_fallback, per-particle mass drift)."""
    nf = ctypes.c_int32()
    drift = np.zeros(ctx.cfg.n_particles)
    _check(load().iewpf_surrogate_window(ctx.h, net.h, _ptr(state), n_model_steps, first_step,
                                         drift_tol, noise_scale, ctypes.byref(nf),
                                         drift.ctypes.data, _stream(stream)))
    return nf.value, drift


def surrogate_window_async(ctx, net, state, n_model_steps: int, first_step: int,
                           drift_tol: float, noise_scale: float, n_fallback_dev, drift_dev=None,
                           stream=None):
    """The window without host waits (capturable): n_fallback_dev is a device int32 tensor
    of one element, drift_dev a device float64 tensor [n_particles] or None."""
    _check(load().iewpf_surrogate_window_async(
        ctx.h, net.h, _ptr(state), n_model_steps, first_step, drift_tol, noise_scale,
        _ptr(n_fallback_dev), _ptr(drift_dev) if drift_dev is not None else None,
        _stream(stream)))


def forecast_drifters_surrogate(ctx, net, state, pos, n_windows: int, steps_per_window: int,
                                first_step: int, drift_tol: float, noise_scale: float, traj=None,
                                stream=None) -> int:
    """Surrogate drifter forecast; returns the number of plain re-steps over all windows."""
    nf = ctypes.c_int32()
    _check(load().iewpf_forecast_drifters_surrogate(
        ctx.h, net.h, _ptr(state), _ptr(pos), int(pos.shape[1]), n_windows, steps_per_window,
        first_step, drift_tol, noise_scale, _ptr(traj), ctypes.byref(nf), _stream(stream)))
    return nf.value
