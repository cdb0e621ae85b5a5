"""ctypes binding of libidmx.so (the C ABI in include/idm.h).

Argument marshalling only: every step of the simulation and its gradient runs
in the library's HIP kernels.  Raises if the library is missing or a call
returns an error status.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libidmx.so")

IDM_OK = 0
STATUS_NAMES = {0: "IDM_OK", -1: "IDM_ERR_INVALID_ARG", -2: "IDM_ERR_LAYOUT",
                -3: "IDM_ERR_UNSUPPORTED", -4: "IDM_ERR_WORKSPACE", -5: "IDM_ERR_HIP"}
BOUND_SOFTPLUS = 0
BOUND_CLAMP = 1

c_int32, c_int64, c_float, c_double = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
c_void_p, c_size_t = ctypes.c_void_p, ctypes.c_size_t


class IdmProblem(ctypes.Structure):
    _fields_ = [("n_vehicles", c_int32), ("n_lanes", c_int32), ("n_steps", c_int32),
                ("ckpt_every", c_int32), ("dt", c_float), ("delta", c_float), ("a_min", c_float),
                ("gap_floor", c_float), ("bound", c_int32), ("lane_offsets_host", c_void_p)]


class IdmTuning(ctypes.Structure):
    _fields_ = [("threads", c_int32), ("per_thread", c_int32), ("ckpt_every", c_int32),
                ("grid", c_int32), ("block", c_int32), ("store_states", c_int32),
                ("tile_steps", c_int32)]


class IdmParams(ctypes.Structure):
    _fields_ = [("v0", c_void_p), ("T", c_void_p), ("a", c_void_p), ("b", c_void_p),
                ("s0", c_void_p), ("length", c_void_p)]


class IdmObs(ctypes.Structure):
    _fields_ = [("target", c_void_p), ("n_obs", c_int32), ("obs_first", c_int32),
                ("obs_stride", c_int32)]


class IdmPlanInfo(ctypes.Structure):
    _fields_ = [("threads", c_int32), ("per_thread", c_int32), ("ckpt_every", c_int32),
                ("grid", c_int32), ("block", c_int32), ("n_bundles", c_int32), ("max_lane", c_int32),
                ("n_slots", c_int64), ("fill", c_double), ("n_levels", c_int32),
                ("n_boundaries", c_int32), ("autotune_cached", c_int32),
                ("store_states", c_int32), ("tile_steps", c_int32)]


class IdmFitState(ctypes.Structure):
    _fields_ = [("u", c_void_p), ("m", c_void_p), ("v", c_void_p), ("params", c_void_p),
                ("length", c_void_p), ("step", c_void_p), ("loss_hist", c_void_p),
                ("hist_len", c_int32), ("lo", c_float * 5), ("hi", c_float * 5),
                ("lr0", c_float), ("lr1", c_float), ("lr_steps", c_int32),
                ("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("raw_units", c_int32)]


class IdmMlpState(ctypes.Structure):
    _fields_ = [("params", c_void_p), ("weights_bf16", c_void_p), ("adam_m", c_void_p),
                ("adam_v", c_void_p), ("lr", c_float), ("beta1", c_float), ("beta2", c_float),
                ("eps", c_float)]


class IdmMlpSchedule(ctypes.Structure):
    _fields_ = [("step", c_void_p), ("lr0", c_float), ("lr_final", c_float),
                ("total_steps", c_int32), ("loss_hist", c_void_p), ("hist_len", c_int32)]


MLP_IN, MLP_IN_PAD, MLP_HIDDEN, MLP_OUT, MLP_OUT_PAD = 150, 160, 256, 5, 16


class IdmEgoProblem(ctypes.Structure):
    _fields_ = [("n_traj", c_int32), ("n_steps", c_int32), ("ckpt_every", c_int32),
                ("dt", c_float), ("delta", c_float), ("a_min", c_float), ("gap_floor", c_float),
                ("bound", c_int32)]


class IdmEgoVars(ctypes.Structure):
    _fields_ = [("v0", c_void_p), ("T", c_void_p), ("a", c_void_p), ("b", c_void_p),
                ("s0", c_void_p), ("gap", c_void_p), ("dv", c_void_p)]


class IdmEgoObs(ctypes.Structure):
    _fields_ = [("offsets", c_void_p), ("step", c_void_p), ("pos", c_void_p), ("n_obs", c_int32)]


class IdmEgoFitState(ctypes.Structure):
    _fields_ = [("params", c_void_p), ("gap", c_void_p), ("dv", c_void_p), ("m", c_void_p),
                ("v", c_void_p), ("step", c_void_p), ("loss_hist", c_void_p),
                ("hist_len", c_int32), ("lo", c_float * 5), ("hi", c_float * 5),
                ("lr0", c_float), ("lr1", c_float), ("lr_steps", c_int32),
                ("beta1", c_float), ("beta2", c_float), ("eps", c_float)]


class IdmStepArgs(ctypes.Structure):
    _fields_ = [("prm", IdmParams), ("p0", c_void_p), ("v_init", c_void_p),
                ("traj_d", c_void_p), ("traj_v", c_void_p),
                ("grad_traj_d", c_void_p), ("grad_traj_v", c_void_p),
                ("obs_target", c_void_p), ("n_obs", c_int32), ("obs_first", c_int32),
                ("obs_stride", c_int32),
                ("grad_params", c_void_p), ("grad_p0", c_void_p), ("grad_v0", c_void_p),
                ("loss_out", c_void_p), ("workspace", c_void_p)]


# every symbol declared in include/idm.h
EXPORTS = ("idm_plan_create", "idm_plan_destroy", "idm_workspace_bytes", "idm_plan_get_info",
           "idm_problem_check", "idm_problem_layout", "idm_problem_bundles",
           "idm_sim_forward", "idm_sim_backward", "idm_sim_backward_stored",
           "idm_sim_backward_noalloc", "idm_plan_diagnostics",
           "idm_fit_init", "idm_fit_step", "idm_fit_run",
           "idm_step_graph_launch", "idm_plan_autotune", "idm_copy_bytes", "idm_last_error",
           "idm_version", "idm_mlp_param_count", "idm_mlp_weight_bf16_count",
           "idm_mlp_workspace_bytes", "idm_mlp_sync", "idm_mlp_features", "idm_mlp_forward",
           "idm_mlp_gradients", "idm_mlp_train_step", "idm_mlp_train_step_scheduled",
           "idm_fit_init_normalized", "idm_observe",
           "idm_lane_loss", "idm_select_by_lane",
           "idm_ego_plan_create", "idm_ego_plan_destroy", "idm_ego_workspace_bytes",
           "idm_ego_match_steps", "idm_ego_initial_speed", "idm_ego_forward", "idm_ego_backward",
           "idm_ego_fit_init", "idm_ego_fit_step", "idm_ego_fit_run")

_lib = None


class IdmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s failed: %s (%s)" % (where, msg, STATUS_NAMES.get(status, status)))
        self.status = status


def load() -> ctypes.CDLL:
    """Load libidmx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libidmx.so not found at %s: run __graft_entry__.build() or "
                          "python paper_2412_16750_amd/build.py" % LIB_PATH)
    # torch first: its wheel carries its own HIP and HSA runtimes under the
    # same sonames as ROCm's, so whichever loads first serves the process.
    # Loading torch's makes this library bind to it, as torch's kernels do;
    # loading this library first would bring in a second HSA runtime next to
    # torch's, after which this library's HIP calls find no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.idm_plan_create.argtypes = [P(IdmProblem), P(IdmTuning), P(c_void_p)]
    L.idm_plan_destroy.argtypes = [c_void_p]
    L.idm_workspace_bytes.argtypes = [c_void_p]
    L.idm_workspace_bytes.restype = c_size_t
    L.idm_plan_get_info.argtypes = [c_void_p, P(IdmPlanInfo)]
    L.idm_problem_check.argtypes = [P(IdmProblem), P(IdmTuning), P(IdmPlanInfo), P(c_size_t)]
    L.idm_problem_layout.argtypes = [P(IdmProblem), P(IdmTuning), c_void_p, c_void_p, c_int64]
    L.idm_problem_bundles.argtypes = [P(IdmProblem), P(IdmTuning), c_void_p, c_void_p, c_void_p,
                                      c_int64]
    L.idm_sim_forward.argtypes = [c_void_p, P(IdmParams), c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p]
    L.idm_sim_backward.argtypes = [c_void_p, P(IdmParams), c_void_p, c_void_p, c_void_p, c_void_p,
                                   P(IdmObs), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p]
    L.idm_sim_backward_stored.argtypes = [c_void_p, P(IdmParams), c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, P(IdmObs), c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p]
    L.idm_sim_backward_noalloc.argtypes = [c_void_p, P(IdmParams), c_void_p, c_void_p, c_void_p,
                                           c_void_p, P(IdmObs), c_void_p, c_void_p, c_void_p,
                                           c_void_p, c_void_p]
    L.idm_plan_diagnostics.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    L.idm_fit_init.argtypes = [c_void_p, P(IdmFitState), c_void_p, c_void_p]
    L.idm_fit_step.argtypes = [c_void_p, P(IdmFitState), c_void_p, c_void_p, P(IdmObs), c_void_p,
                               c_void_p]
    L.idm_fit_run.argtypes = [c_void_p, P(IdmFitState), c_void_p, c_void_p, P(IdmObs), c_int32,
                              c_void_p, c_void_p]
    L.idm_step_graph_launch.argtypes = [c_void_p, P(IdmStepArgs), c_void_p]
    L.idm_plan_autotune.argtypes = [c_void_p, P(IdmStepArgs), c_size_t, c_int32, c_void_p]
    L.idm_copy_bytes.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    L.idm_copy_bytes.restype = c_int32
    L.idm_mlp_param_count.restype = c_int64
    L.idm_mlp_weight_bf16_count.restype = c_int64
    L.idm_mlp_workspace_bytes.argtypes = [c_int64]
    L.idm_mlp_workspace_bytes.restype = c_size_t
    L.idm_mlp_sync.argtypes = [P(IdmMlpState), c_void_p]
    L.idm_mlp_features.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                   c_void_p, c_void_p]
    L.idm_mlp_forward.argtypes = [P(IdmMlpState), c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    L.idm_mlp_gradients.argtypes = [P(IdmMlpState), c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                    c_void_p, c_void_p]
    L.idm_mlp_train_step.argtypes = [P(IdmMlpState), c_void_p, c_void_p, c_int64, c_int32, c_void_p,
                                     c_void_p, c_void_p]
    L.idm_mlp_train_step_scheduled.argtypes = [P(IdmMlpState), c_void_p, c_void_p, c_int64,
                                               c_void_p, c_int64, P(IdmMlpSchedule), c_void_p,
                                               c_void_p, c_void_p, c_void_p]
    L.idm_fit_init_normalized.argtypes = [c_void_p, P(IdmFitState), c_void_p, c_int32, c_void_p]
    L.idm_observe.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                              c_void_p, c_void_p]
    L.idm_lane_loss.argtypes = [c_void_p, c_void_p, c_void_p, P(IdmObs), c_void_p, c_void_p]
    L.idm_select_by_lane.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p]
    for name in ("idm_mlp_sync", "idm_mlp_features", "idm_mlp_forward", "idm_mlp_gradients",
                 "idm_mlp_train_step", "idm_mlp_train_step_scheduled", "idm_fit_init_normalized",
                 "idm_observe", "idm_lane_loss",
                 "idm_select_by_lane"):
        getattr(L, name).restype = c_int32
    L.idm_ego_plan_create.argtypes = [P(IdmEgoProblem), P(c_void_p)]
    L.idm_ego_plan_destroy.argtypes = [c_void_p]
    L.idm_ego_workspace_bytes.argtypes = [c_void_p]
    L.idm_ego_workspace_bytes.restype = c_size_t
    L.idm_ego_match_steps.argtypes = [c_void_p, c_int32, c_double, c_int32, c_void_p, c_void_p]
    L.idm_ego_initial_speed.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]
    L.idm_ego_forward.argtypes = [c_void_p, P(IdmEgoVars), c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p]
    L.idm_ego_backward.argtypes = [c_void_p, P(IdmEgoVars), c_void_p, P(IdmEgoObs), c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.idm_ego_fit_init.argtypes = [c_void_p, P(IdmEgoFitState), P(c_float * 5), c_float, c_float,
                                   c_void_p]
    L.idm_ego_fit_step.argtypes = [c_void_p, P(IdmEgoFitState), c_void_p, P(IdmEgoObs), c_void_p,
                                   c_void_p]
    L.idm_ego_fit_run.argtypes = [c_void_p, P(IdmEgoFitState), c_void_p, P(IdmEgoObs), c_int32,
                                  c_void_p, c_void_p]
    for name in ("idm_ego_plan_create", "idm_ego_plan_destroy", "idm_ego_match_steps",
                 "idm_ego_initial_speed", "idm_ego_forward", "idm_ego_backward", "idm_ego_fit_init",
                 "idm_ego_fit_step", "idm_ego_fit_run"):
        getattr(L, name).restype = c_int32
    L.idm_last_error.restype = ctypes.c_char_p
    L.idm_version.restype = ctypes.c_char_p
    for name in ("idm_problem_check", "idm_problem_layout", "idm_problem_bundles", "idm_plan_create",
                 "idm_plan_destroy", "idm_plan_get_info", "idm_sim_forward",
                 "idm_sim_backward", "idm_sim_backward_stored", "idm_sim_backward_noalloc",
                 "idm_plan_diagnostics",
                 "idm_fit_init", "idm_fit_step",
                 "idm_fit_run", "idm_step_graph_launch",
                 "idm_plan_autotune"):
        getattr(L, name).restype = c_int32
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != IDM_OK:
        msg = load().idm_last_error().decode(errors="replace")
        raise IdmError(status, where, msg)
