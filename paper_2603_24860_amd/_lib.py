"""ctypes declarations of the C ABI in include/bse.h.

The shared library must exist (built by build_lib.build()); importing this
module without it raises immediately -- there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbse.so")

OK, EINVAL, ESHAPE, EWORKSPACE, EDEVICE, ENOCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16X3 = 0, 1, 2
GROUP_OH, GROUP_D6H = 0, 1

i32, i64, u8, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint8, ctypes.c_double
vp = ctypes.c_void_p
P = ctypes.POINTER


class BseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bse status {status}: {msg}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("grid", i32 * 3), ("nk", i32), ("nops", i32), ("nkorb", i32),
                ("nporb", i32), ("ncls", i32)]


class Tables(ctypes.Structure):
    _fields_ = [("kperm", vp), ("korb", vp), ("korb_rep", vp), ("porb", vp), ("porb_rep", vp),
                ("pidx", vp), ("pconj", vp), ("cls_rep", vp), ("cls_selfswap", vp)]


class BlockDims(ctypes.Structure):
    _fields_ = [("n", i64), ("nmem", i32), ("nub", i64)]


class Problem(ctypes.Structure):
    _fields_ = [("grid", i32 * 3), ("nv", i32), ("nc", i32), ("nmb", i32),
                ("nkorb", i32), ("ncls", i32), ("nqorb", i32),
                ("korb", vp), ("qorb", vp), ("pidx", vp), ("pconj", vp),
                ("ev", vp), ("ec", vp), ("vdiag", vp),
                ("mx", vp), ("mv", vp), ("mc", vp), ("w", vp), ("in_fp64", i32)]


class Block(ctypes.Structure):
    _fields_ = [("n", i64), ("mem_off", vp), ("members", vp), ("orb_off", vp),
                ("orb_dim", vp), ("ub_off", vp), ("ubasis", vp)]


def _load():
    # PyTorch ships its own HIP runtime with the same SONAME (libamdhip64.so.7)
    # as the ROCm one libbse.so is linked against.  Loading torch first makes
    # the library bind to that runtime, so kernels launched here and the torch
    # allocations and streams they use live in one HIP runtime instance.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_24860_amd.build_lib`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "bse_last_error": (ctypes.c_char_p, []),
        "bse_version": (ctypes.c_char_p, []),
        "bse_group_order": (i32, [i32]),
        "bse_group_nirreps": (i32, [i32]),
        "bse_group_ops": (i32, [i32, vp, vp]),
        "bse_group_irrep": (i32, [i32, i32, ctypes.c_char_p, P(i32), vp]),
        "bse_dims_get": (i32, [i32, vp, P(Dims)]),
        "bse_tables_build": (i32, [i32, vp, P(Tables)]),
        "bse_block_dims_get": (i32, [i32, vp, i32, i32, i32, P(BlockDims)]),
        "bse_block_basis": (i32, [i32, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "bse_partner_block_dims_get": (i32, [i32, vp, i32, i32, i32, i32, P(BlockDims)]),
        "bse_partner_block_basis": (i32, [i32, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "bse_build_ws": (ctypes.c_size_t, [P(Problem), i32]),
        "bse_build_ws_min": (ctypes.c_size_t, [P(Problem), i32]),
        "bse_build": (i32, [P(Problem), i32, vp, i64, vp, ctypes.c_size_t, vp]),
        "bse_seed_ws": (ctypes.c_size_t, [i32, P(Problem), i32]),
        "bse_seed_plan": (i32, [i32, P(Problem), i32, vp, ctypes.c_size_t, P(i64), vp]),
        "bse_build_seed": (i32, [i64, vp, i64, vp]),
        "bse_project_seed": (i32, [i64, i32, P(Block), P(vp), P(i64), vp]),
        "bse_seed_free": (i32, [i64]),
        "bse_project_blocks": (i32, [P(Problem), vp, i64, i32, vp, i32, P(Block),
                                     P(vp), P(i64), P(vp), vp]),
        "bse_dipole_weights": (i32, [P(Problem), vp, i32, P(Block), vp, vp, vp]),
        "bse_block_eigh_ws": (ctypes.c_size_t, [i64, i32, i32, i32]),
        "bse_block_eigh_set_two_stage": (i64, [i64]),
        "bse_block_eigh": (i32, [i64, vp, i64, i32, vp, i32, i32, vp, vp, vp, vp,
                                 ctypes.c_size_t, vp]),
        "bse_block_eigh_status": (i32, [i64, i32, i32, vp, P(i32), vp]),
        "bse_block_eigh_noalloc_max": (ctypes.c_size_t, []),
        "bse_block_eigh_noalloc": (i32, [i64, vp, i64, i32, vp, i32, i32, vp, vp, vp, vp]),
        "bse_batch_eigh_ws": (ctypes.c_size_t, [i32, P(i64), i32, i32]),
        "bse_batch_eigh_plan": (i32, [i32, P(i64), P(vp), P(i64), i32, P(vp), i32, P(vp), P(vp),
                                      P(vp), vp, ctypes.c_size_t, P(i64), vp]),
        "bse_batch_eigh_run": (i32, [i64, vp]),
        "bse_batch_eigh_tune": (i32, [i64, vp, P(i32), P(i32)]),
        "bse_batch_eigh_config": (i32, [i64, i32, i32, vp]),
        "bse_batch_eigh_free": (i32, [i64]),
        "bse_spectrum": (i32, [i64, vp, vp, f64, f64, i64, vp, vp, vp]),
        "bse_eels_ws": (ctypes.c_size_t, [i64]),
        "bse_eels": (i32, [i64, vp, vp, f64, vp, vp, vp, ctypes.c_size_t, vp]),
        "bse_haydock_ws": (ctypes.c_size_t, [i64]),
        "bse_haydock": (i32, [i64, vp, i64, i32, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]),
        "bse_haydock_spectrum": (i32, [i32, vp, vp, f64, f64, i64, vp, vp, vp]),
        "bse_sync_probe": (i32, [i32, i32, i32, vp, P(f64), vp]),
        "bse_prof_enable": (i32, [ctypes.c_char_p]),
        "bse_prof_collect": (i32, []),
        "bse_prof_count": (i32, []),
        "bse_prof_get": (i32, [i32, ctypes.c_char_p, P(f64), P(i64)]),
        "bse_prof_reset": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib, sorted(sig)


lib, EXPORTS = _load()


def check(status):
    if status < 0:
        raise BseError(status, lib.bse_last_error().decode())
    return status
