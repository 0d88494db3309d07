"""ctypes declarations of the C ABI in include/mlbm.h (argument marshalling only).

The shared library is loaded from the package directory; a missing library is
an error (there is no fallback implementation).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlbm.so")

MLBM_OK = 0
MLBM_ERR_ARG = -1
MLBM_ERR_GEOMETRY = -2
MLBM_ERR_SINGULAR = -3
MLBM_ERR_HIP = -4
MLBM_ERR_UNSUPPORTED = -5
MLBM_ERR_UNSTABLE = -6

FLUID, WALL, DIRICHLET = 0, 1, 2
FLAG_LAGRANGE = 0x400
POPULATIONS, FIELDS = 0, 1
F64, F32, F16S, BF16 = 0, 1, 2, 3

RED_MASS, RED_INT_UX, RED_INT_UY, RED_INT_SPEED, RED_NORM_U2, RED_NORM_DU2 = range(6)
RED_FORCE_X, RED_FORCE_Y, RED_N_BAD, RED_FIRST_BAD = 6, 7, 8, 9
RED_RESIDUAL, RED_PREV_INT_UX, RED_MEAN_CHANGE, RED_PERMEABILITY, RED_COUNT = 10, 11, 12, 13, 14
STEADY_FIELD, STEADY_MEAN = 0, 1
STATIC_MAX_NODES = 1 << 24

_p = ctypes.c_void_p


class Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xy", _p), ("kind", _p),
                ("lo", ctypes.c_double * 2), ("hi", ctypes.c_double * 2),
                ("periodic", ctypes.c_int32 * 2), ("wall_lo_y", ctypes.c_int32),
                ("wall_hi_y", ctypes.c_int32), ("n_disks", ctypes.c_int64), ("disks", _p),
                ("fluid_area", ctypes.c_double)]


class StencilParams(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("reorder", ctypes.c_int32), ("dx", ctypes.c_double),
                ("n_threads", ctypes.c_int32), ("lattice_h", ctypes.c_double),
                ("per_departure", ctypes.c_int32), ("simple_bounce_back", ctypes.c_int32)]


class Stencils(ctypes.Structure):
    _fields_ = [("perm", _p), ("idx", _p), ("w", _p), ("bb", _p), ("area", _p), ("lagrange", _p),
                ("w_lagrange", _p), ("n_lagrange", ctypes.c_int64)]


class Sizes(ctypes.Structure):
    _fields_ = [("idx_bytes", ctypes.c_int64), ("w_bytes", ctypes.c_int64),
                ("flags_bytes", ctypes.c_int64), ("state_bytes", ctypes.c_int64),
                ("k_padded", ctypes.c_int32)]


class StepParams(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("tau_plus", ctypes.c_double), ("tau_minus", ctypes.c_double),
                ("g", ctypes.c_double * 2), ("scale_exp", ctypes.c_int32),
                ("block", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("fp32_arith", ctypes.c_int32), ("alternate_sweeps", ctypes.c_int32),
                ("cached_weights", ctypes.c_int32), ("stochastic_rounding", ctypes.c_int32),
                ("weights16", ctypes.c_int32), ("hybrid_launches", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("lanes_per_node", ctypes.c_int32)]


class DeviceState(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("K", ctypes.c_int32), ("idx", _p), ("w", _p),
                ("flags", _p), ("bc", _p), ("state", _p * 2), ("cur", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("max_halo", ctypes.c_int32), ("halo_off", _p),
                ("halo", _p), ("lidx", _p), ("w_lagrange", _p), ("lagrange_begin", ctypes.c_int64),
                ("step_count", ctypes.c_uint64), ("per_departure", ctypes.c_int32)]


class Steady(ctypes.Structure):
    _fields_ = [("criterion", ctypes.c_int32), ("check_every", ctypes.c_int32), ("hold", ctypes.c_int32),
                ("max_steps", ctypes.c_int64), ("tol", ctypes.c_double)]


class Batch(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("check_every", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("sample_tile_off", _p), ("sample_tile_off_host", _p), ("area", _p), ("u_prev", _p),
                ("tile_red", _p), ("queue", _p), ("counters", _p), ("sample_steps", _p),
                ("sample_residual", _p), ("sample_int_ux", _p), ("n_groups", ctypes.c_int32),
                ("group_sample_off", _p), ("group_sample_off_host", _p), ("group_queue_off", _p)]


class ConvDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("c_in", ctypes.c_int32), ("c_out", ctypes.c_int32), ("ksize", ctypes.c_int32),
                ("x_stride", ctypes.c_int32), ("x_offset", ctypes.c_int32),
                ("y_stride", ctypes.c_int32), ("y_offset", ctypes.c_int32), ("c_store", ctypes.c_int32)]


class UNetDesc(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("channels", ctypes.c_int32 * 6), ("batch", ctypes.c_int32),
                ("res", ctypes.c_int32), ("c_in", ctypes.c_int32), ("c_out", ctypes.c_int32),
                ("params", _p), ("grads", _p), ("adam_m", _p), ("adam_v", _p), ("w_bf16", _p), ("act", _p),
                ("act_grad", _p), ("work", _p)]


class UNetBuffers(ctypes.Structure):
    _fields_ = [("n_params", ctypes.c_int64), ("w_bf16_bytes", ctypes.c_int64), ("act_bytes", ctypes.c_int64),
                ("work_bytes", ctypes.c_int64), ("n_layers", ctypes.c_int32)]


class UNetLayerInfo(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 8), ("ksize", ctypes.c_int32), ("c_in", ctypes.c_int32),
                ("c_out", ctypes.c_int32), ("res", ctypes.c_int32), ("w_offset", ctypes.c_int64),
                ("b_offset", ctypes.c_int64)]


class MlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mlbm error {code}: {msg}")
        self.code = code


def _load():
    # One HIP runtime per process: when PyTorch is present its runtime is the
    # process's, and the library must bind to that same libamdhip64 (same
    # soname) rather than load a second copy, so PyTorch is imported first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "python paper_2312_14789_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "mlbm_build_stencils": (ctypes.c_int, [P(Geometry), P(StencilParams), P(Stencils)]),
        "mlbm_packed_sizes": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, P(Sizes)]),
        "mlbm_pack_stencils": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _p, _p,
                                              _p, _p, _p, _p, _p]),
        "mlbm_pack_stencils_range": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                                    ctypes.c_int32, ctypes.c_int32, _p, _p, _p, _p, _p,
                                                    _p, _p]),
        "mlbm_mark_lagrange": (ctypes.c_int, [ctypes.c_int64, _p, _p]),
        "mlbm_weights_to_f16": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, _p, _p]),
        "mlbm_batch_init": (ctypes.c_int, [P(StepParams), P(DeviceState), P(Batch), _p]),
        "mlbm_step_batched": (ctypes.c_int, [P(StepParams), P(DeviceState), P(Batch), ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_int32, P(ctypes.c_int32), _p]),
        "mlbm_tile_sizes": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _p,
                                           P(ctypes.c_int64), P(ctypes.c_int32)]),
        "mlbm_pack_tiles": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _p, _p, _p, _p]),
        "mlbm_init_state": (ctypes.c_int, [P(StepParams), P(DeviceState), _p, _p, _p]),
        "mlbm_step": (ctypes.c_int, [P(StepParams), P(DeviceState), ctypes.c_int32, _p]),
        "mlbm_reduction_workspace_bytes": (ctypes.c_int64, [ctypes.c_int64]),
        "mlbm_macroscopic": (ctypes.c_int, [P(StepParams), P(DeviceState), _p, ctypes.c_double,
                                            ctypes.c_double, _p, _p, _p, _p, _p, _p]),
        "mlbm_reductions_reset": (ctypes.c_int, [_p, _p]),
        "mlbm_macroscopic_static": (ctypes.c_int, [P(StepParams), P(DeviceState), _p, ctypes.c_double,
                                                   ctypes.c_double, _p, _p, _p, _p, _p]),
        "mlbm_run_to_steady": (ctypes.c_int, [P(StepParams), P(DeviceState), P(Steady), _p, ctypes.c_double,
                                              ctypes.c_double, _p, _p, _p, _p, P(ctypes.c_int64), _p]),
        "mlbm_conv_forward": (ctypes.c_int, [P(ConvDesc), _p, _p, _p, _p, ctypes.c_int32, ctypes.c_int32, _p]),
        "mlbm_conv_wgrad_workspace": (ctypes.c_int64, [P(ConvDesc), ctypes.c_int32]),
        "mlbm_conv_wgrad": (ctypes.c_int, [P(ConvDesc), _p, _p, _p, _p, ctypes.c_int32, _p, _p]),
        "mlbm_conv_weights": (ctypes.c_int, [_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _p, _p, _p]),
        "mlbm_relu_backward": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, _p, ctypes.c_int32, ctypes.c_int32,
                                              _p, ctypes.c_int32, ctypes.c_int32, _p]),
        "mlbm_pool_forward": (ctypes.c_int, [ctypes.c_int32] * 4 + [_p, ctypes.c_int32, ctypes.c_int32, _p,
                                                                     ctypes.c_int32, ctypes.c_int32, _p]),
        "mlbm_pool_backward": (ctypes.c_int, [ctypes.c_int32] * 4 + [_p, ctypes.c_int32, ctypes.c_int32, _p,
                                                                      ctypes.c_int32, ctypes.c_int32, _p,
                                                                      ctypes.c_int32, ctypes.c_int32, _p]),
        "mlbm_upsample_forward": (ctypes.c_int, [ctypes.c_int32] * 4 + [_p, ctypes.c_int32, ctypes.c_int32, _p,
                                                                         ctypes.c_int32, ctypes.c_int32, _p]),
        "mlbm_upsample_backward": (ctypes.c_int, [ctypes.c_int32] * 4 + [_p, ctypes.c_int32, ctypes.c_int32, _p,
                                                                          ctypes.c_int32, ctypes.c_int32, _p]),
        "mlbm_mse_workspace": (ctypes.c_int64, [ctypes.c_int64]),
        "mlbm_masked_mse": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, _p, ctypes.c_int32, _p, _p,
                                           ctypes.c_float, _p, _p, _p, _p]),
        "mlbm_adam": (ctypes.c_int, [ctypes.c_int64, _p, _p, _p, _p, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_int32, _p]),
        "mlbm_unet_sizes": (ctypes.c_int, [P(UNetDesc), P(UNetBuffers)]),
        "mlbm_unet_layer": (ctypes.c_int, [P(UNetDesc), ctypes.c_int32, P(UNetLayerInfo)]),
        "mlbm_unet_refresh": (ctypes.c_int, [P(UNetDesc), _p]),
        "mlbm_unet_forward": (ctypes.c_int, [P(UNetDesc), _p, _p, _p]),
        "mlbm_unet_loss": (ctypes.c_int, [P(UNetDesc), _p, _p, _p, _p, _p]),
        "mlbm_unet_backward": (ctypes.c_int, [P(UNetDesc), _p, _p]),
        "mlbm_unet_adam": (ctypes.c_int, [P(UNetDesc), ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_int32, _p]),
        "mlbm_last_error": (ctypes.c_char_p, []),
        "mlbm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()

# every symbol the header declares (checked by the tests)
EXPORTS = ["mlbm_build_stencils", "mlbm_packed_sizes", "mlbm_pack_stencils", "mlbm_pack_stencils_range",
           "mlbm_mark_lagrange", "mlbm_weights_to_f16",
           "mlbm_tile_sizes", "mlbm_pack_tiles", "mlbm_init_state", "mlbm_batch_init", "mlbm_step_batched",
           "mlbm_step", "mlbm_reduction_workspace_bytes", "mlbm_reductions_reset", "mlbm_macroscopic", "mlbm_macroscopic_static",
           "mlbm_run_to_steady", "mlbm_last_error", "mlbm_version"]

# every symbol include/mlbm_unet.h declares
UNET_EXPORTS = ["mlbm_unet_sizes", "mlbm_unet_layer", "mlbm_unet_refresh", "mlbm_unet_forward", "mlbm_unet_loss",
                "mlbm_unet_backward", "mlbm_unet_adam", "mlbm_conv_forward", "mlbm_conv_wgrad_workspace", "mlbm_conv_wgrad", "mlbm_conv_weights",
                "mlbm_relu_backward", "mlbm_pool_forward", "mlbm_pool_backward", "mlbm_upsample_forward",
                "mlbm_upsample_backward", "mlbm_mse_workspace", "mlbm_masked_mse", "mlbm_adam"]


def check(rc):
    if rc != MLBM_OK:
        raise MlbmError(rc, lib.mlbm_last_error().decode())
    return rc
