"""ctypes declarations of the C ABI in include/pbn.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbn_amd.so")

MAX_PAIRS = 64

OK, EINVAL, ENOMEM, ELIMIT, ELDS, EHIP, ERANGE, ENODEV = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ELIMIT: "ELIMIT", ELDS: "ELDS", EHIP: "EHIP",
          ERANGE: "ERANGE", ENODEV: "ENODEV"}


class PbnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class pbn_desc(C.Structure):
    _fields_ = [("n", C.c_uint32), ("p", C.c_double),
                ("fn_off", C.POINTER(C.c_uint32)), ("sel_prob", C.POINTER(C.c_double)),
                ("par_off", C.POINTER(C.c_uint32)), ("parents", C.POINTER(C.c_uint32)),
                ("tt_off", C.POINTER(C.c_uint32)), ("tt", C.POINTER(C.c_uint64))]


class pbn_plan_opts(C.Structure):
    _fields_ = [("reduce", C.c_uint32), ("group", C.c_uint32), ("weight_mode", C.c_uint32),
                ("lds_budget_bytes", C.c_uint32), ("theta", C.c_uint64),
                ("max_table_entries", C.c_uint32), ("max_parent_bits", C.c_uint32),
                ("max_group_nodes", C.c_uint32), ("sampling", C.c_uint32),
                ("state_bits", C.c_uint32), ("reserved", C.c_uint32)]


class pbn_plan_info(C.Structure):
    _fields_ = [(name, C.c_uint32) for name in (
        "n", "n_kept", "n_slots", "n_table_slots", "n_passes", "state_words", "n_jobs",
        "image_bytes", "table_bytes", "image_in_lds", "blob_bytes", "max_fn_parents",
        "max_union_bits", "n_multi_groups", "state_bytes")] + [("reserved", C.c_uint32 * 5)]


class pbn_targets(C.Structure):
    _fields_ = [("ntargets", C.c_uint32), ("npairs", C.c_uint32),
                ("pos", C.c_uint32 * MAX_PAIRS), ("val", C.c_uint32 * MAX_PAIRS),
                ("mask", C.c_uint64 * 64)]


class pbn_launch_opts(C.Structure):
    _fields_ = [("waves_per_block", C.c_uint32), ("record_traj", C.c_uint32), ("record_words", C.c_uint32),
                ("traj_per_wave", C.c_uint32), ("d_record", C.c_void_p)]


class pbn_rl_out(C.Structure):
    _fields_ = [("k", C.c_uint32), ("reserved", C.c_uint32), ("g2", C.c_double), ("bic", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("burn_in", C.c_double),
                ("n_required", C.c_double), ("p_hat", C.c_double), ("steps", C.c_uint64)]


class pbn_skart_out(C.Structure):
    _fields_ = [("done", C.c_uint32), ("stage", C.c_uint32), ("n_required", C.c_uint64),
                ("batch_size", C.c_uint64), ("batch_count", C.c_uint32), ("spacer", C.c_uint32),
                ("failures", C.c_uint32), ("ci_batches", C.c_uint32), ("ci_batch_size", C.c_uint64),
                ("warmup", C.c_uint64), ("p_hat", C.c_double), ("lower", C.c_double), ("upper", C.c_double),
                ("half_width", C.c_double), ("skewness", C.c_double), ("lag1", C.c_double),
                ("ar_factor", C.c_double), ("steps", C.c_uint64)]


class pbn_work(C.Structure):
    _fields_ = [("d_plan", C.c_void_p), ("d_targets", C.c_void_p), ("d_state", C.c_void_p),
                ("d_counts", C.c_void_p), ("seed", C.c_uint64), ("traj0", C.c_uint32),
                ("ntraj", C.c_uint32), ("count_from", C.c_uint32), ("step0", C.c_uint32)]


class pbn_estimate_out(C.Structure):
    _fields_ = [("p_hat", C.c_double), ("half_width", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("n_required", C.c_double), ("burn_in", C.c_double),
                ("units", C.c_uint32), ("reserved", C.c_uint32)]


_lib = None

# name -> (restype, argtypes)
_P = C.c_void_p
_U32, _U64, _SZ = C.c_uint32, C.c_uint64, C.c_size_t
_pU32, _pU64, _pI32 = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_int32)
SIGNATURES = {
    "pbn_last_error": (C.c_char_p, []),
    "pbn_net_create": (C.c_int32, [C.POINTER(pbn_desc), C.POINTER(_P)]),
    "pbn_net_destroy": (C.c_int32, [_P]),
    "pbn_net_tables": (C.c_int32, [_P, _pU64, _pU64, _pI32]),
    "pbn_plan_opts_default": (None, [C.POINTER(pbn_plan_opts)]),
    "pbn_plan_build": (C.c_int32, [_P, _pU32, _U32, C.POINTER(pbn_plan_opts), C.POINTER(_P)]),
    "pbn_plan_destroy": (C.c_int32, [_P]),
    "pbn_plan_info_get": (C.c_int32, [_P, C.POINTER(pbn_plan_info)]),
    "pbn_plan_node_pos": (C.c_int32, [_P, _pU32]),
    "pbn_plan_slots": (C.c_int32, [_P, _pU32, _pU32]),
    "pbn_plan_alg4_groups": (C.c_int32, [_P, _pU32, _pU32, _pU32, _pU32]),
    "pbn_plan_single_groups": (C.c_int32, [_P, _pU32, _pU32, _pU32, _pU32]),
    "pbn_eq2_lower_bound": (C.c_int32, [_pU64, _U32, _U64, _pU32]),
    "pbn_plan_export": (C.c_int32, [_P, _P, C.POINTER(_SZ)]),
    "pbn_targets_build": (C.c_int32, [_P, _pU32, _pU32, _pU32, _U32, _U32, C.POINTER(pbn_targets)]),
    "pbn_state_init": (C.c_int32, [_P, _P, _U64, _U32, _U32, _P, _P]),
    "pbn_simulate": (C.c_int32, [_P, _P, _U64, _U32, _U32, _U32, _U32, _U32,
                                 C.POINTER(pbn_targets), _P, _P, C.POINTER(pbn_launch_opts), _P]),
    "pbn_simulate_plain": (C.c_int32, [_P, _P, _U64, _U32, _U32, _U32, _U32, _U32,
                                       C.POINTER(pbn_targets), _P, _P, C.POINTER(pbn_launch_opts), _P]),
    "pbn_state_to_original": (C.c_int32, [_P, _P, _P, _U32, _P, _P]),
    "pbn_batch_tasks": (C.c_int32, [C.POINTER(_P), _pU32, _U32, _U32, _U32, _pU32, _pU32, _pU32, _pU32]),
    "pbn_batch_launch": (C.c_int32, [C.POINTER(_P), _U32, _P, _P, _P, _U32, _pU32, _U32, _P, _U32, _U32, _P]),
    "pbn_batch_launch_noalloc": (C.c_int32, [C.POINTER(_P), _pU32, _U32, _P, _U32, _U32, _U32, _P]),
    "pbn_probe_lds_gather": (C.c_int32, [_U32, _U32, _U32, _U32, _U32, _P, _P]),
    "pbn_probe_vmem_gather": (C.c_int32, [_P, _U32, _U32, _U32, _U32, _U32, _P, _P]),
    "pbn_batch_graph_create": (C.c_int32, [C.POINTER(_P), _U32, _P, _P, _P, _U32, _pU32, _U32, _P, _U32, _U32,
                                           _U32, C.POINTER(_P)]),
    "pbn_graph_launch": (C.c_int32, [_P, _P]),
    "pbn_graph_destroy": (C.c_int32, [_P]),
    "pbn_estimate": (C.c_int32, [_pU64, _U32, _U64, C.c_double, C.c_double, C.POINTER(pbn_estimate_out)]),
    "pbn_skart_analyze": (C.c_int32, [_pU32, _U64, C.c_double, C.c_double, C.POINTER(pbn_skart_out)]),
    "pbn_skart_run": (C.c_int32, [_P, _P, _U64, _U32, C.POINTER(pbn_targets), _P, _P, _P, _U32, C.c_double,
                                  C.c_double, _U64, C.POINTER(pbn_launch_opts), C.POINTER(pbn_skart_out), _P]),
    "pbn_rl_diagnose": (C.c_int32, [_pU32, _U64, C.c_double, C.c_double, C.c_double, _U32,
                                    C.POINTER(pbn_rl_out)]),
    "pbn_rl_run": (C.c_int32, [_P, _P, _U64, _U32, C.POINTER(pbn_targets), _P, _P, _P, _U32, C.c_double,
                               C.c_double, C.c_double, _U32, _U64, _U64, C.POINTER(pbn_launch_opts),
                               C.POINTER(pbn_rl_out), _P]),
    "pbn_t_quantile": (C.c_double, [C.c_double, C.c_double]),
    "pbn_normal_quantile": (C.c_double, [C.c_double]),
}


def lib():
    """The loaded library.  Raises if it was not built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != OK:
        msg = lib().pbn_last_error().decode(errors="replace")
        raise PbnError(code, msg)
    return code
