"""ctypes declarations of the libddf C ABI (include/ddf.h).

The shared library is built in-tree (``paper_1908_06742_amd/libddf.so``) by
``paper_1908_06742_amd.build``.  Loading fails loudly when it is missing: there is
no CPU fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddf.so")

DDF_F64, DDF_F32, DDF_F16, DDF_BF16, DDF_BF16_SR = 0, 1, 2, 3, 4
STORAGE = {"f64": DDF_F64, "f32": DDF_F32, "f16": DDF_F16, "bf16": DDF_BF16, "bf16sr": DDF_BF16_SR}
STORAGE_BYTES = {DDF_F64: 8, DDF_F32: 4, DDF_F16: 2, DDF_BF16: 2, DDF_BF16_SR: 2}

DDF_OK, DDF_ERR_ARG, DDF_ERR_UNSUPPORTED, DDF_ERR_HIP, DDF_ERR_NONFINITE, DDF_ERR_STATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "DDF_OK", -1: "DDF_ERR_ARG", -2: "DDF_ERR_UNSUPPORTED", -3: "DDF_ERR_HIP",
                -4: "DDF_ERR_NONFINITE", -5: "DDF_ERR_STATE"}

FORCE = {"none": 0, "uniform": 1, "fourroll": 2, "pulsatile": 3}
LAYOUT = {"auto": 0, "row": 1, "interleaved": 2, "packed": 3}
LAYOUT_NAMES = {1: "row", 2: "interleaved", 3: "packed"}
SCALAR = {"mrt": 0, "srt": 1, "cascaded": 2, "central": 3}

OUTPUTS = ("rho", "ux", "uy", "phi", "Sxx", "Syy", "Sxy", "wz",
           "dxuy", "dyux", "dxphi", "dyphi", "Q", "R", "Lx", "Ly")
STATS = ("mass", "scalar", "res_u", "res_phi", "nonfinite", "steps", "umax", "phimin")


class DDFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("storage", C.c_int32), ("scalar_model", C.c_int32),
        ("omega", C.c_double * 9), ("omega_phi", C.c_double * 9),
        ("beta1", C.c_double), ("beta2", C.c_double),
        ("cs2", C.c_double), ("cs2_phi", C.c_double),
        ("wall_u", (C.c_double * 2) * 4),
        ("wall_phi", C.c_double * 4),
        ("force_kind", C.c_int32), ("layout", C.c_int32),
        ("force", C.c_double * 2),
        ("force_k", C.c_double), ("force_omega", C.c_double),
        ("rho0", C.c_double), ("phi0", C.c_double),
        ("pop_scale", C.c_double), ("phi_min", C.c_double),
    ]


# Every symbol include/ddf.h declares, with (restype, argtypes).
_vp = C.c_void_p
_P = C.POINTER(Params)
SIGNATURES = {
    "ddf_pitch": (C.c_int64, [_P]),
    "ddf_plane_stride": (C.c_int64, [_P]),
    "ddf_population_bytes": (C.c_size_t, [_P]),
    "ddf_workspace_bytes": (C.c_size_t, [_P]),
    "ddf_create": (C.c_int, [_P, _vp, _vp, _vp, C.POINTER(_vp)]),
    "ddf_destroy": (None, [_vp]),
    "ddf_init_equilibrium": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "ddf_step": (C.c_int, [_vp, C.c_int64, _vp]),
    "ddf_extract": (C.c_int, [_vp, _vp, C.c_uint32, C.c_int32, _vp]),
    "ddf_reduce": (C.c_int, [_vp, C.POINTER(C.c_double), _vp]),
    "ddf_get_populations": (C.c_int, [_vp, _vp, _vp, C.c_int32, _vp]),
    "ddf_set_populations": (C.c_int, [_vp, _vp, _vp, C.c_int32, C.c_int64, _vp]),
    "ddf_step_count": (C.c_int64, [_vp]),
    "ddf_get_layout": (C.c_int32, [_vp]),
    "ddf_set_tile_width": (C.c_int, [_vp, C.c_int32]),
    "ddf_get_tile_width": (C.c_int32, [_vp]),
    "ddf_set_address_width": (C.c_int, [_vp, C.c_int32]),
    "ddf_get_address_width": (C.c_int32, [_vp]),
    "ddf_set_workgroups_per_cu": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "ddf_get_workgroups_per_cu": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ddf_set_graph": (C.c_int, [_vp, C.c_int32]),
    "ddf_last_error": (C.c_char_p, []),
    "ddf_batch_population_bytes": (C.c_size_t, [C.c_int32, _P]),
    "ddf_batch_workspace_bytes": (C.c_size_t, [C.c_int32, _P]),
    "ddf_batch_create": (C.c_int, [C.c_int32, _P, _vp, _vp, _vp, C.POINTER(_vp)]),
    "ddf_batch_destroy": (None, [_vp]),
    "ddf_batch_size": (C.c_int32, [_vp]),
    "ddf_batch_step_count": (C.c_int64, [_vp]),
    "ddf_batch_offsets": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "ddf_batch_init_equilibrium": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "ddf_batch_set_tiling": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "ddf_batch_get_tiling": (C.c_int, [_vp] + [C.POINTER(C.c_int32)] * 4),
    "ddf_batch_set_nontemporal": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "ddf_batch_get_nontemporal": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ddf_batch_autotune": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_float), _vp]),
    "ddf_batch_set_graph": (C.c_int, [_vp, C.c_int32]),
    "ddf_batch_set_active": (C.c_int, [_vp, C.POINTER(C.c_uint8)]),
    "ddf_batch_init_instance": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "ddf_batch_step": (C.c_int, [_vp, C.c_int64, _vp]),
    "ddf_batch_reduce": (C.c_int, [_vp, C.POINTER(C.c_double), _vp]),
    "ddf_batch_step_reduce": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.c_void_p]),
    "ddf_batch_extract": (C.c_int, [_vp, C.c_int32, _vp, C.c_uint32, C.c_int32, _vp]),
    "ddf_batch_get_populations": (C.c_int, [_vp, C.c_int32, _vp, _vp, C.c_int32, _vp]),
}

# Surrogate-network kernels (include/ddf_nn.h).
_i32, _i64, _f32 = C.c_int32, C.c_int64, C.c_float
_fp = C.POINTER(C.c_float)
_dp = C.POINTER(C.c_double)
NN_CAST_MAX_LAYERS = 32


class CastLayer(C.Structure):
    """ddf_nn_cast_layer (include/ddf_nn.h)."""
    _fields_ = [("w", C.c_void_p), ("wf", C.c_void_p), ("wd", C.c_void_p),
                ("Cout", C.c_int32), ("Cin", C.c_int32), ("Cout_p", C.c_int32), ("Cin_p", C.c_int32)]


NN_SIGNATURES = {
    "ddf_nn_conv3x3": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32,
                                 _vp, _i32, _i32, _vp]),
    "ddf_nn_wgrad_workspace_bytes": (C.c_size_t, [_i32, _i32, _i32, _i32, _i32, C.POINTER(_i32)]),
    "ddf_nn_conv3x3_wgrad": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _vp, _i32,
                                       _vp, _vp]),
    "ddf_nn_relu_bwd": (C.c_int, [_vp, _vp, _i64, _vp]),
    "ddf_nn_pool2": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp]),
    "ddf_nn_pool2_bwd": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _i32, _vp]),
    "ddf_nn_up2": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp]),
    "ddf_nn_up2_bwd": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp]),
    "ddf_nn_slice": (C.c_int, [_vp, _i32, _i32, _vp, _i32, _i32, _i64, _i32, _i32, _vp]),
    "ddf_nn_mse_workspace_bytes": (C.c_size_t, [_i64]),
    "ddf_nn_mse": (C.c_int, [_vp, _i32, _vp, _i64, _fp, _vp, _vp, _vp, _vp]),
    "ddf_nn_mse_static_max_pixels": (C.c_size_t, []),
    "ddf_nn_mse_static": (C.c_int, [_vp, _i32, _vp, _i64, _fp, _vp, _vp, _vp]),
    "ddf_nn_adam": (C.c_int, [_vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _i64, _f32, _vp]),
    "ddf_nn_cast_weights": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "ddf_nn_cast_weights_multi": (C.c_int, [_i32, C.POINTER(CastLayer), _vp]),
    "ddf_nn_cavity_inputs": (C.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _f32, _f32, _f32, _vp, _vp]),
    "ddf_nn_cavity_targets": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp]),
    "ddf_nn_cavity_fields": (C.c_int, [_vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
}
SIGNATURES.update(NN_SIGNATURES)

# include/ddf_probe.h
PROBE_COPY, PROBE_READ, PROBE_WRITE = 0, 1, 2
SIGNATURES["ddf_bandwidth_probe"] = (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _vp, _vp, C.c_size_t, _vp])
SIGNATURES["ddf_pattern_probe"] = (C.c_int, [_vp, C.c_int32, C.c_int32, _vp])
SIGNATURES["ddf_batch_pattern_probe"] = (C.c_int, [_vp, C.c_int32, _vp])

_lib = None


def lib():
    """The loaded libddf.so.  Raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libddf.so not found at {LIB_PATH}; build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != DDF_OK:
        raise DDFError(rc, lib().ddf_last_error().decode())
    return rc


def params_from_problem(pr) -> Params:
    """Marshal a problem description (attributes of workloads.Problem) into ddf_params."""
    p = Params()
    p.nx, p.ny = int(pr.nx), int(pr.ny)
    p.periodic_x, p.periodic_y = int(bool(pr.periodic_x)), int(bool(pr.periodic_y))
    p.storage = STORAGE[pr.storage]
    p.scalar_model = SCALAR[pr.scalar_model]
    w = 1.0 / pr.tau
    p.omega[:] = [0.0, 0.0, 0.0, pr.omega3, w, w] + list(pr.omega_hi)
    wp = 1.0 / pr.tau_phi
    p.omega_phi[:] = [0.0, wp, wp] + list(pr.omega_phi_hi)
    p.beta1, p.beta2 = pr.beta1, pr.beta2
    p.cs2, p.cs2_phi = pr.cs2, pr.cs2phi
    for s in range(4):
        p.wall_u[s][0] = pr.wall_u[s][0]
        p.wall_u[s][1] = pr.wall_u[s][1]
    p.wall_phi[:] = [float("nan") if v is None else float(v) for v in pr.wall_phi]
    p.force_kind = FORCE[pr.force_kind]
    p.force[:] = list(pr.force)
    p.force_k = pr.force_k
    p.force_omega = pr.force_omega
    p.rho0, p.phi0 = pr.rho0, pr.phi0
    p.pop_scale = getattr(pr, "pop_scale", 0.0) or 0.0
    p.phi_min = pr.phi_min
    p.layout = LAYOUT[getattr(pr, "layout", "auto")]
    return p
