"""ctypes declarations of the C ABI in include/pflb.h and include/pfsur.h."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpflb.so")

OK = 0
ERRORS = {-1: "PFLB_ERR_PARAM", -2: "PFLB_ERR_ALIGN", -3: "PFLB_ERR_UNBOUND",
          -4: "PFLB_ERR_DEVICE", -5: "PFLB_ERR_NONFINITE", -6: "PFLB_ERR_IO",
          -7: "PFLB_ERR_NOMEM"}
ERR_NONFINITE = -5

BC_PERIODIC, BC_WALL = 0, 1
STORE_FP32, STORE_FP16S, STORE_FP32_INPLACE = 0, 1, 2
NBUF = 3


class PflbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("bc", ctypes.c_int * 3),
                ("rho_L", ctypes.c_double), ("rho_H", ctypes.c_double),
                ("nu_L", ctypes.c_double), ("nu_H", ctypes.c_double),
                ("M", ctypes.c_double), ("W", ctypes.c_double), ("sigma", ctypes.c_double),
                ("g", ctypes.c_double * 3),
                ("eps", ctypes.c_double),
                ("hoc", ctypes.c_int),
                ("dtheta_C", ctypes.c_double),
                ("storage", ctypes.c_int),
                ("scale_log2", ctypes.c_int * 2),
                ("wall_u", ctypes.c_double * 18),
                ("wet_cos", ctypes.c_double * 6),
                ("open", ctypes.c_int * 6),
                ("open_P", ctypes.c_double * 6)]


class LayerIO(ctypes.Structure):
    _fields_ = [("in_off", ctypes.c_size_t), ("out_off", ctypes.c_size_t),
                ("pool_off", ctypes.c_size_t),
                ("in_cs", ctypes.c_int), ("in_c0", ctypes.c_int), ("in_mode", ctypes.c_int),
                ("out_cs", ctypes.c_int), ("out_c0", ctypes.c_int), ("pool_cs", ctypes.c_int),
                ("Cin", ctypes.c_int), ("Cout", ctypes.c_int), ("level", ctypes.c_int)]


class SurCfg(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("in_shift", ctypes.c_float * 4), ("in_scale", ctypes.c_float * 4),
                ("out_scale", ctypes.c_float * 4), ("lrr_scale", ctypes.c_float)]


_vp = ctypes.c_void_p
_SIGS = {
    "pflb_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(_vp)]),
    "pflb_destroy": (None, [_vp]),
    "pflb_last_error": (ctypes.c_char_p, [_vp]),
    "pflb_required_bytes": (ctypes.c_size_t, [ctypes.POINTER(Params), ctypes.c_int]),
    "pflb_bind": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int]),
    "pflb_equilibrium": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pflb_set_state": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pflb_get_state": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pflb_init_fields": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pflb_init_fields_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "pflb_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "pflb_reconstruct": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "pflb_step": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "pflb_step_graph": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "pflb_step_many": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp]),
    "pflb_read": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pflb_mass": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int), _vp]),
    "pflb_step_count": (ctypes.c_longlong, [_vp]),
    "pflb_save": (ctypes.c_int, [_vp, ctypes.c_char_p, _vp]),
    "pflb_load": (ctypes.c_int, [_vp, ctypes.c_char_p, _vp]),
    # surrogate
    "pfsur_num_params": (ctypes.c_size_t, []),
    "pfsur_create": (ctypes.c_int, [ctypes.POINTER(SurCfg), ctypes.POINTER(_vp)]),
    "pfsur_destroy": (None, [_vp]),
    "pfsur_last_error": (ctypes.c_char_p, [_vp]),
    "pfsur_set_params": (ctypes.c_int, [_vp, _vp]),
    "pfsur_get_params": (ctypes.c_int, [_vp, _vp]),
    "pfsur_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SurCfg), ctypes.c_int, ctypes.c_int]),
    "pfsur_layer_io_of": (ctypes.c_int, [ctypes.POINTER(SurCfg), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(LayerIO)]),
    "pfsur_pack": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.c_int, _vp, _vp]),
    "pfsur_pack_target": (ctypes.c_int, [_vp] * 7 + [ctypes.POINTER(ctypes.c_double),
                                                    ctypes.c_int, _vp, _vp]),
    "pfsur_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "pfsur_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int, _vp]),
    "pfsur_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                        ctypes.POINTER(ctypes.c_float), _vp, _vp]),
    "pfsur_gradients": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp,
                                       ctypes.POINTER(ctypes.c_float), _vp, _vp]),
    "pfsur_guard_work_bytes": (ctypes.c_size_t, [ctypes.POINTER(SurCfg), ctypes.c_int]),
    "pflb_advance_guarded": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int), _vp, _vp]),
    "pflb_advance_guarded_trace": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int,
                                                  ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_double), _vp, _vp]),
    "pfsur_guard_accept": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double]),
    "pfsur_conv_fwd": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp,
                                      _vp, _vp]),
    "pfsur_conv_wgrad_work_bytes": (ctypes.c_size_t, [ctypes.c_int] * 5),
    "pfsur_conv_wgrad": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                        _vp]),
    "pfsur_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "pfsur_load": (ctypes.c_int, [_vp, ctypes.c_char_p]),
}

_lib = None


def load_library(path=LIB_PATH, build_if_missing=True):
    """Load libpflb.so (building it first only if no built library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        if not build_if_missing:
            raise OSError(f"{path} is not built")
        from .build_lib import build
        build()
    so = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(so, name)
        fn.restype = res
        fn.argtypes = args
    _lib = so
    return so


def lib():
    return load_library()


def exported_symbols():
    return list(_SIGS)
