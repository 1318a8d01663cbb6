"""ctypes declarations of libsymten's C ABI (include/symten.h)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SYMTEN_LIB selects another build of the same library (the host-sanitized one)
LIB_PATH = os.environ.get("SYMTEN_LIB") or os.path.join(HERE, "libsymten.so")

OK = 0
ERRORS = {-1: "E_INVAL", -2: "E_LEGS", -3: "E_SYM", -4: "E_NOMEM", -5: "E_HIP",
          -6: "E_LINALG", -7: "E_CAPACITY", -8: "E_UNSUPPORTED", -9: "E_NODEVICE"}
U1, SU2, Z2 = 1, 2, 3
F64, F32 = 0, 1
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3, "bf16x6": 4}
MAX_SECTORS = 64


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class SymtenError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [("group", C.c_int), ("rank", C.c_int), ("dirs", C.POINTER(C.c_int)),
                ("nsec", C.POINTER(C.c_int)), ("labels", C.POINTER(C.c_int)),
                ("dims", C.POINTER(C.c_int)), ("flux", C.c_int), ("dtype", C.c_int)]


class PlanStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("pairs", "out_blocks", "useful_flops", "groups",
                                         "gemm_flops", "max_m", "max_n", "max_k")]

    def to_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class MoveStats(C.Structure):
    _fields_ = [("nsec", C.c_int), ("charge", C.c_int * MAX_SECTORS), ("kept", C.c_int * MAX_SECTORS),
                ("n_sv_sectors", C.c_int), ("sv_charge", C.c_int * MAX_SECTORS),
                ("sv_count", C.c_int * MAX_SECTORS),
                ("trunc_err", C.c_double), ("gap", C.c_double), ("s_max", C.c_double), ("cutoff", C.c_double),
                ("flops_corners", C.c_int64), ("flops_halves", C.c_int64), ("flops_renorm", C.c_int64),
                ("flops_proj", C.c_int64),
                ("ms_corners", C.c_double), ("ms_halves", C.c_double), ("ms_proj", C.c_double),
                ("ms_renorm", C.c_double), ("ms_total", C.c_double)]

    def to_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if not n.startswith(("charge", "kept", "sv_"))}
        d["kept"] = {int(self.charge[i]): int(self.kept[i]) for i in range(self.nsec)}
        d["sv_sectors"] = {int(self.sv_charge[i]): int(self.sv_count[i]) for i in range(self.n_sv_sectors)}
        d.pop("nsec")
        d.pop("n_sv_sectors")
        return d


class RunOpts(C.Structure):
    _fields_ = [("chi", C.c_int), ("chi_max", C.c_int), ("prec", C.c_int), ("block", C.c_int),
                ("max_steps", C.c_int), ("tol", C.c_double)]


class RunResult(C.Structure):
    _fields_ = [("kappa", C.c_double), ("err_steps", C.c_double), ("err_chi", C.c_double),
                ("error", C.c_double), ("steps", C.c_int), ("total_steps", C.c_int), ("chi", C.c_int),
                ("levels", C.c_int)]

    def to_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 64), ("launches", C.c_int64), ("ms", C.c_double),
                ("useful_flops", C.c_int64), ("gemm_flops", C.c_int64), ("bytes", C.c_int64)]

    def to_dict(self):
        return {"name": self.name.decode(), "launches": int(self.launches), "ms": float(self.ms),
                "useful_flops": int(self.useful_flops), "gemm_flops": int(self.gemm_flops),
                "bytes": int(self.bytes)}


_lib = None
P = C.c_void_p
H = C.c_void_p
I64P = C.POINTER(C.c_int64)
IP = C.POINTER(C.c_int)

SIGNATURES = {
    "symten_create": (C.c_int, [C.POINTER(H), C.POINTER(Desc), P]),
    "symten_create_meta": (C.c_int, [C.POINTER(H), C.POINTER(Desc)]),
    "symten_destroy": (None, [H]),
    "symten_rank": (C.c_int, [H, IP]),
    "symten_flux": (C.c_int, [H, IP]),
    "symten_dtype": (C.c_int, [H, IP]),
    "symten_leg_info": (C.c_int, [H, C.c_int, IP, IP, IP, IP]),
    "symten_num_blocks": (C.c_int, [H, I64P]),
    "symten_nnz": (C.c_int, [H, I64P]),
    "symten_block_info": (C.c_int, [H, C.c_int64, IP, IP, I64P, I64P]),
    "symten_block_tree": (C.c_int, [H, C.c_int64, IP, IP]),
    "symten_su2_to_u1": (C.c_int, [C.POINTER(H), H, P]),
    "symten_su2_cg": (C.c_int, [C.c_int] * 6 + [C.POINTER(C.c_double)]),
    "symten_device_ptr": (C.c_int, [H, C.POINTER(P), I64P]),
    "symten_nbytes": (C.c_int, [H, I64P]),
    "symten_set_allocator": (C.c_int, [P, P, P]),
    "symten_upload": (C.c_int, [H, C.POINTER(C.c_double), C.c_int64, P]),
    "symten_download": (C.c_int, [H, C.POINTER(C.c_double), C.c_int64, P]),
    "symten_contract": (C.c_int, [C.POINTER(H), H, H, C.c_int, IP, IP, IP, C.c_int, P]),
    "symten_contract_noalloc": (C.c_int, [H, H, H, C.c_int, IP, IP, IP, C.c_int, P]),
    "symten_match_blocks": (C.c_int, [H, H, C.c_int, IP, IP, P, C.c_int64, P, C.c_int64, P, P]),
    "symten_plan_info": (C.c_int, [H, H, C.c_int, IP, IP, IP, C.POINTER(PlanStats), C.POINTER(H)]),
    "symten_double_layer": (C.c_int, [C.POINTER(H), H, P]),
    "symten_enlarged_corner": (C.c_int, [C.POINTER(H), C.c_int, H, H, H, H, C.c_int,
                                         C.POINTER(PlanStats), P]),
    "symten_enlarged_corner_single_layer": (C.c_int, [C.POINTER(H), C.c_int, H, H, H, H, C.c_int,
                                                      C.POINTER(PlanStats), P]),
    "symten_enlarged_corners_batched": (C.c_int, [C.c_int, C.POINTER(H), C.POINTER(H), C.POINTER(H),
                                                  C.POINTER(H), C.POINTER(H), C.c_int, C.c_int,
                                                  C.POINTER(PlanStats), P]),
    "ctm_env_create": (C.c_int, [C.POINTER(H), C.POINTER(H), C.POINTER(H)]),
    "ctm_env_destroy": (None, [H]),
    "ctm_env_get": (C.c_int, [H, C.c_int, C.POINTER(H)]),
    "ctm_move": (C.c_int, [H, H, C.c_int, C.c_int, C.c_int, C.POINTER(MoveStats), P]),
    "ctm_site_partition": (C.c_int, [H, H, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), P]),
    "ctm_run": (C.c_int, [H, H, C.POINTER(RunOpts), C.POINTER(RunResult), P]),
    "ctm_expectation": (C.c_int, [H, H, C.c_int, C.c_int, C.POINTER(H), C.POINTER(C.c_double), P]),
    "ctm_heisenberg_bond_energy": (C.c_int, [H, H, C.POINTER(C.c_double), C.POINTER(C.c_double), P]),
    "symten_double_layer_op": (C.c_int, [C.POINTER(H), H, C.POINTER(C.c_double), P]),
    "ctm_cell_create": (C.c_int, [C.POINTER(H), C.c_int, C.c_int, C.POINTER(H), C.POINTER(H)]),
    "ctm_cell_get": (C.c_int, [H, C.c_int, C.c_int, C.c_int, C.POINTER(H)]),
    "ctm_cell_move": (C.c_int, [H, C.POINTER(H), C.c_int, C.c_int, C.c_int, P]),
    "ctm_cell_site_partition": (C.c_int, [H, C.c_int, C.c_int, H, C.c_int, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), P]),
    "ctm_move_singular_values": (C.c_int, [H, C.POINTER(C.c_double), C.c_int64, I64P]),
    "ctm_move_projectors": (C.c_int, [H, C.POINTER(H), C.POINTER(H)]),
    "ctm_env_set": (C.c_int, [H, C.c_int, H]),
    "symten_eigh": (C.c_int, [C.c_int, IP, C.POINTER(P), IP, C.POINTER(P), IP, C.POINTER(P), P]),
    "symten_eigh_max_order": (C.c_int, [IP]),
    "symten_profile_begin": (C.c_int, []),
    "symten_profile_end": (C.c_int, [C.POINTER(KernelStat), C.c_int, IP]),
    "symten_last_error": (C.c_char_p, []),
    "symten_version": (C.c_int, []),
    "symten_sync": (C.c_int, [P]),
}


def lib():
    """Load libsymten.so; raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: when torch is present it has already
        # loaded libamdhip64/rocBLAS/rocSOLVER (same sonames), and libsymten
        # must bind to those so that torch's streams and memory are valid in it.
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_1808_10804_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        msg = lib().symten_last_error()
        raise SymtenError(rc, msg.decode() if msg else "")
    return rc
