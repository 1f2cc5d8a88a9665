"""ctypes view of libpdmp.so (include/pdmp.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdmp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pdmp.h")

PDMP_OK, PDMP_EINVAL, PDMP_EUNSUPPORTED, PDMP_EDEVICE, PDMP_ENOMEM = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "PDMP_OK", 1: "PDMP_EINVAL", 2: "PDMP_EUNSUPPORTED", 3: "PDMP_EDEVICE",
                4: "PDMP_ENOMEM"}
MAX_DOF = 8


class pdmp_occupancy(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_hinges", C.c_int32), ("hinges", C.c_void_p),
                ("weights", C.c_void_p), ("lengthscale", C.c_float), ("grid", C.c_int32 * 3)]


class pdmp_arm(C.Structure):
    _fields_ = [("n_dof", C.c_int32), ("pts_per_link", C.c_int32),
                ("a", C.c_float * MAX_DOF), ("d", C.c_float * MAX_DOF),
                ("alpha", C.c_float * MAX_DOF), ("theta0", C.c_float * MAX_DOF)]


class pdmp_discs(C.Structure):
    _fields_ = [("n", C.c_int32), ("centres", C.c_void_p), ("radii", C.c_void_p)]


class pdmp_boxes(C.Structure):
    _fields_ = [("n", C.c_int32), ("centres", C.c_void_p), ("half", C.c_void_p)]


class pdmp_fit_opts(C.Structure):
    _fields_ = [("optimizer", C.c_int32), ("steps", C.c_int32), ("lr", C.c_float),
                ("lr_bias", C.c_float), ("l2", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("t0", C.c_int32),
                ("adam_m", C.c_void_p), ("adam_v", C.c_void_p)]


class pdmp_mlp(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("hidden", C.c_int32), ("n_hidden", C.c_int32),
                ("params", C.c_void_p), ("params_bf16", C.c_void_p)]


class pdmp_tanh_net(C.Structure):
    _fields_ = [("dim", C.c_int32), ("hidden", C.c_int32), ("n_hidden", C.c_int32),
                ("params", C.c_void_p)]


class pdmp_sampler_opts(C.Structure):
    _fields_ = [("dim", C.c_int32), ("T", C.c_int32), ("eta", C.c_float), ("batch", C.c_int64),
                ("capacity", C.c_int64), ("seed", C.c_uint64), ("stream_id", C.c_uint32),
                ("prior_stream_id", C.c_uint32), ("lo", C.c_float * 3), ("hi", C.c_float * 3)]


class pdmp_sampler_stats(C.Structure):
    _fields_ = [("batches", C.c_int64), ("produced", C.c_int64), ("popped_bucket", C.c_int64),
                ("popped_prior", C.c_int64), ("bucket_size", C.c_int64), ("status", C.c_int32),
                ("running", C.c_int32), ("producer_busy_s", C.c_double),
                ("elapsed_s", C.c_double)]


class pdmp_rrt_opts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("step", C.c_float), ("goal_tol", C.c_float),
                ("start", C.c_float * 2), ("goal", C.c_float * 2), ("time_budget_s", C.c_double),
                ("n_discs", C.c_int32), ("disc_x", C.c_void_p), ("disc_y", C.c_void_p),
                ("disc_r", C.c_void_p)]


class pdmp_rrt_result(C.Structure):
    _fields_ = [("solved", C.c_int32), ("iters", C.c_int32), ("n_nodes", C.c_int32),
                ("from_bucket", C.c_int64), ("from_prior", C.c_int64), ("path_len", C.c_double),
                ("elapsed_s", C.c_double)]


class pdmp_cull_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("lo", C.c_float * 3), ("inv_cell", C.c_float),
                ("nc", C.c_int32 * 3)]


_vp, _i32, _i64, _u32, _u64, _f = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
_P = C.POINTER

# name -> (restype, argtypes); every symbol declared in include/pdmp.h
SIGNATURES = {
    "pdmp_abi_version": (_i32, []),
    "pdmp_last_error": (C.c_char_p, []),
    "pdmp_sync": (_i32, [_vp]),
    "pdmp_uniform_samples": (_i32, [_u64, _u32, _P(_f), _P(_f), _i32, _i64, _vp, _vp]),
    "pdmp_label_points_discs": (_i32, [_P(pdmp_discs), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_label_points_boxes": (_i32, [_P(pdmp_boxes), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_label_configs": (_i32, [_P(pdmp_arm), _P(pdmp_boxes), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_occupancy_eval": (_i32, [_P(pdmp_occupancy), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_occupancy_grad": (_i32, [_P(pdmp_occupancy), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_morph_samples": (_i32, [_P(pdmp_occupancy), _P(pdmp_arm), _vp, _vp, _i64, _i32, _f, _vp]),
    "pdmp_occupancy_bwd_noalloc": (_i32, [_P(pdmp_occupancy), _vp, _i64, _vp, _vp, _vp, _vp,
                                          _vp]),
    "pdmp_morph_workspace_size": (C.c_size_t, [_P(pdmp_occupancy), _P(pdmp_arm), _i64, _i32]),
    "pdmp_morph_samples_ws": (_i32, [_P(pdmp_occupancy), _P(pdmp_arm), _vp, _vp, _i64, _i32, _f,
                                     _vp, C.c_size_t, _vp]),
    "pdmp_split_scheme": (_i32, [_P(pdmp_occupancy), _P(_i32), _vp]),
    "pdmp_tanh_split_scheme": (_i32, [_P(pdmp_tanh_net), _P(_i32), _vp]),
    "pdmp_issue_rates": (_i32, [_P(C.c_double), _i32]),
    "pdmp_morph_trajectory": (_i32, [_P(pdmp_occupancy), _P(pdmp_arm), _vp, _vp, _i64, _i32, _f,
                                     _vp, _i64, _vp]),
    "pdmp_fk_body_points": (_i32, [_P(pdmp_arm), _vp, _i64, _vp, _vp]),
    "pdmp_fit_workspace_size": (C.c_size_t, [_i32, _i32, _i64]),
    "pdmp_bwd_workspace_size": (C.c_size_t, [_i32, _i32, _i64]),
    "pdmp_bce_workspace_size": (C.c_size_t, [_i64]),
    "pdmp_fit_occupancy": (_i32, [_P(pdmp_occupancy), _vp, _vp, _vp, _i64, _P(pdmp_fit_opts), _vp,
                                  _vp, C.c_size_t, _vp]),
    "pdmp_occupancy_bwd": (_i32, [_P(pdmp_occupancy), _vp, _i64, _vp, _vp, _vp, _vp, _vp,
                                  C.c_size_t, _vp]),
    "pdmp_bce_logits": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "pdmp_adam_step": (_i32, [_vp, _vp, _vp, _vp, _i64, _i64, _i32, _f, _f, _f, _f, _f, _vp]),
    "pdmp_mlp_num_params": (_i64, [_P(pdmp_mlp)]),
    "pdmp_cull_grid_make": (_i32, [_i32, _P(_f), _P(_f), _f, _P(pdmp_cull_grid)]),
    "pdmp_morph_culled_workspace_size": (C.c_size_t, [_P(pdmp_occupancy), _P(pdmp_cull_grid),
                                                      _i64]),
    "pdmp_morph_culled": (_i32, [_P(pdmp_occupancy), _P(pdmp_cull_grid), _vp, _vp, _i64, _i32, _f,
                                 _vp, C.c_size_t, _vp]),
    "pdmp_bucket_create": (_i32, [_i32, _i64, _P(_vp)]),
    "pdmp_bucket_push": (_i64, [_vp, _vp, _i64, _i64, _i64, _i64]),
    "pdmp_bucket_pop": (_i32, [_vp, _vp, _vp]),
    "pdmp_bucket_size": (_i64, [_vp]),
    "pdmp_bucket_destroy": (None, [_vp]),
    "pdmp_sampler_create": (_i32, [_P(pdmp_occupancy), _P(pdmp_sampler_opts), _P(_vp)]),
    "pdmp_sampler_start": (_i32, [_vp]),
    "pdmp_sampler_pause": (_i32, [_vp, _i32]),
    "pdmp_sampler_pop": (_i32, [_vp, _i64, _vp, _vp, _vp]),
    "pdmp_sampler_get_stats": (_i32, [_vp, _P(pdmp_sampler_stats)]),
    "pdmp_sampler_destroy": (_i32, [_vp]),
    "pdmp_rrt_run": (_i32, [_vp, _P(pdmp_rrt_opts), _vp, _vp, _vp, _vp, _vp,
                            _P(pdmp_rrt_result)]),
    "pdmp_morph_logdet": (_i32, [_P(pdmp_occupancy), _vp, _vp, _i64, _i32, _f, _vp, _vp]),
    "pdmp_morph_inverse": (_i32, [_P(pdmp_occupancy), _vp, _vp, _i64, _i32, _f, _i32, _vp, _vp,
                                  _vp]),
    "pdmp_morph_logdet_ws": (_i32, [_P(pdmp_occupancy), _vp, _vp, _i64, _i32, _f, _vp, _vp,
                                    C.c_size_t, _vp]),
    "pdmp_morph_inverse_ws": (_i32, [_P(pdmp_occupancy), _vp, _vp, _i64, _i32, _f, _i32, _vp,
                                     _vp, _vp, C.c_size_t, _vp]),
    "pdmp_mixture_samples": (_i32, [_P(pdmp_occupancy), _u64, _u32, _P(_f), _P(_f), _i64, _f,
                                    _i32, _f, _vp, _vp, _vp, _vp]),
    "pdmp_tanh_num_params": (_i64, [_P(pdmp_tanh_net)]),
    "pdmp_tanh_occupancy_eval": (_i32, [_P(pdmp_tanh_net), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_tanh_occupancy_grad": (_i32, [_P(pdmp_tanh_net), _vp, _i64, _vp, _vp, _vp]),
    "pdmp_tanh_morph_samples": (_i32, [_P(pdmp_tanh_net), _vp, _vp, _i64, _i32, _f, _vp]),
    "pdmp_tanh_fit_workspace_size": (C.c_size_t, [_P(pdmp_tanh_net), _i64]),
    "pdmp_tanh_loss_grad": (_i32, [_P(pdmp_tanh_net), _vp, _vp, _i64, _f, _vp, _vp, _vp,
                                   C.c_size_t, _vp]),
    "pdmp_tanh_fit": (_i32, [_P(pdmp_tanh_net), _vp, _vp, _i64, _P(pdmp_fit_opts), _vp, _vp,
                             C.c_size_t, _vp]),
    "pdmp_mlp_pack": (_i32, [_P(pdmp_mlp), _vp, _vp]),
    "pdmp_mlp_acts_size": (C.c_size_t, [_P(pdmp_mlp), _i64]),
    "pdmp_mlp_workspace_size": (C.c_size_t, [_P(pdmp_mlp), _i64]),
    "pdmp_mlp_forward": (_i32, [_P(pdmp_mlp), _vp, _i64, _vp, _vp, _vp, C.c_size_t, _vp]),
    "pdmp_mlp_backward": (_i32, [_P(pdmp_mlp), _vp, _vp, _i64, _vp, _vp, _vp, _vp, C.c_size_t,
                                 _vp]),
    "pdmp_mlp_backward_weighted": (_i32, [_P(pdmp_mlp), _vp, _vp, _i64, _vp, _f, _vp, _vp, _vp,
                                          _vp, C.c_size_t, _vp]),
    "pdmp_arm_max_occupancy": (_i32, [_P(pdmp_occupancy), _P(pdmp_arm), _vp, _i64, _f, _vp, _vp,
                                      _vp]),
    "pdmp_amortised_workspace_size": (C.c_size_t, [_P(pdmp_mlp), _P(pdmp_arm), _i64]),
    "pdmp_amortised_morph": (_i32, [_P(pdmp_mlp), _P(pdmp_occupancy), _P(pdmp_arm), _vp, _vp, _i64,
                                    _i32, _f, _f, _vp, _vp, _vp, C.c_size_t, _vp]),
    "pdmp_amortised_morph_refine": (_i32, [_P(pdmp_mlp), _P(pdmp_occupancy), _P(pdmp_arm), _vp,
                                           _vp, _i64, _i32, _f, _f, _vp, _vp, _vp, C.c_size_t,
                                           _vp]),
}

_lib = None


class PdmpError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load the HIP library; raise loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libpdmp.so not found at {LIB_PATH}: build it first "
            "(python -c 'import __graft_entry__ as g; g.build()' or "
            "python paper_2108_11775_amd/build.py).  There is no CPU fallback.")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def call(name, *args):
    lib = load()
    st = getattr(lib, name)(*args)
    if st != PDMP_OK:
        msg = lib.pdmp_last_error()
        raise PdmpError(name, st, msg.decode() if msg else "")
    return st
