"""Python binding of the C ABI (include/bse.h): argument marshalling only.

Every function here converts numpy arrays or torch tensors into the pointers
and sizes the C entry points take, calls the library, and raises BseError on a
non-OK status.  All arithmetic of the hot path runs in the library's kernels.
PyTorch provides device memory and the current HIP stream.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import BseError, FP32, FP64, BF16X3, GROUP_OH, GROUP_D6H, check, lib  # noqa: F401

GROUPS = {"Oh": GROUP_OH, "D6h": GROUP_D6H}


def _ptr(a):
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def _gid(group):
    return GROUPS[group] if isinstance(group, str) else int(group)


def _grid(grid):
    return np.ascontiguousarray(np.asarray(grid, dtype=np.int32))


# --------------------------------------------------------------------------
# groups and tables (host)
# --------------------------------------------------------------------------
def bse_group_ops(group):
    g = _gid(group)
    n = check(lib.bse_group_order(g))
    kmat = np.zeros((n, 3, 3), dtype=np.int32)
    rcart = np.zeros((n, 3, 3), dtype=np.float64)
    check(lib.bse_group_ops(g, _ptr(kmat), _ptr(rcart)))
    return kmat, rcart


def bse_group_irreps(group):
    g = _gid(group)
    n = check(lib.bse_group_order(g))
    out = []
    for i in range(check(lib.bse_group_nirreps(g))):
        name = ctypes.create_string_buffer(8)
        dim = ctypes.c_int32()
        chi = np.zeros(n)
        check(lib.bse_group_irrep(g, i, name, ctypes.byref(dim), _ptr(chi)))
        out.append((name.value.decode(), dim.value, chi))
    return out


def irrep_index(group, name):
    for i, (nm, _, _) in enumerate(bse_group_irreps(group)):
        if nm == name:
            return i
    raise KeyError(name)


def bse_dims_get(group, grid):
    d = _lib.Dims()
    g = _grid(grid)
    check(lib.bse_dims_get(_gid(group), _ptr(g), ctypes.byref(d)))
    return dict(grid=tuple(d.grid), nk=d.nk, nops=d.nops, nkorb=d.nkorb, nporb=d.nporb,
                ncls=d.ncls)


def bse_tables_build(group, grid):
    d = bse_dims_get(group, grid)
    nk = d["nk"]
    t = dict(kperm=np.zeros((d["nops"], nk), np.int32), korb=np.zeros(nk, np.int32),
             korb_rep=np.zeros(d["nkorb"], np.int32), porb=np.zeros(nk * nk, np.int32),
             porb_rep=np.zeros(d["nporb"], np.int32), pidx=np.zeros(nk * nk, np.int32),
             pconj=np.zeros(nk * nk, np.uint8), cls_rep=np.zeros(d["ncls"], np.int32),
             cls_selfswap=np.zeros(d["ncls"], np.uint8))
    s = _lib.Tables(*[_ptr(t[f]) for f, _ in _lib.Tables._fields_])
    g = _grid(grid)
    check(lib.bse_tables_build(_gid(group), _ptr(g), ctypes.byref(s)))
    t.update(d)
    return t


def bse_block_basis(group, grid, irrep, nv, nc, partner=None):
    """Isotypic block basis of `irrep`, or (partner = p) the partner-resolved
    basis of row p of a vector irrep."""
    g = _grid(grid)
    gid = _gid(group)
    ir = irrep_index(group, irrep) if isinstance(irrep, str) else int(irrep)
    bd = _lib.BlockDims()
    if partner is None:
        check(lib.bse_block_dims_get(gid, _ptr(g), ir, nv, nc, ctypes.byref(bd)))
    else:
        check(lib.bse_partner_block_dims_get(gid, _ptr(g), ir, int(partner), nv, nc,
                                             ctypes.byref(bd)))
    nkorb = bse_dims_get(group, grid)["nkorb"]
    out = dict(n=bd.n, mem_off=np.zeros(nkorb + 1, np.int32), members=np.zeros(bd.nmem, np.int32),
               orb_off=np.zeros(nkorb, np.int64), orb_dim=np.zeros(nkorb, np.int32),
               ub_off=np.zeros(nkorb + 1, np.int64), ubasis=np.zeros(max(bd.nub, 1), np.float64))
    args = [_ptr(out["mem_off"]), _ptr(out["members"]), _ptr(out["orb_off"]),
            _ptr(out["orb_dim"]), _ptr(out["ub_off"]), _ptr(out["ubasis"])]
    if partner is None:
        check(lib.bse_block_basis(gid, _ptr(g), ir, nv, nc, *args))
    else:
        check(lib.bse_partner_block_basis(gid, _ptr(g), ir, int(partner), nv, nc, *args))
    return out


# --------------------------------------------------------------------------
# device entry points
# --------------------------------------------------------------------------
def bse_build_ws(problem, prec):
    return lib.bse_build_ws(ctypes.byref(problem), prec)


def bse_build_ws_min(problem, prec):
    return lib.bse_build_ws_min(ctypes.byref(problem), prec)


def bse_build(problem, prec, H, ws, stream=None):
    """H: complex tensor (N x N, complex128 for FP64 else complex64) on the GPU."""
    ldh = H.stride(0)
    nbytes = ws.numel() * ws.element_size()
    check(lib.bse_build(ctypes.byref(problem), prec, _ptr(H), ldh, _ptr(ws), nbytes,
                        _stream(stream)))


def bse_seed_ws(group, problem, prec):
    return lib.bse_seed_ws(_gid(group), ctypes.byref(problem), prec)


def bse_seed_plan(group, problem, prec, ws, stream=None):
    plan = ctypes.c_int64()
    check(lib.bse_seed_plan(_gid(group), ctypes.byref(problem), prec, _ptr(ws),
                            ws.numel() * ws.element_size(), ctypes.byref(plan), _stream(stream)))
    return plan.value


def bse_build_seed(plan, H, stream=None):
    """H None: the seed pieces only (for bse_project_seed)."""
    check(lib.bse_build_seed(plan, _ptr(H), H.stride(0) if H is not None else 0, _stream(stream)))


def bse_project_seed(plan, blocks, Hmu, stream=None):
    """H_mu of each block straight from the plan's seed pieces (no H)."""
    nb = len(blocks)
    arr = (_lib.Block * max(nb, 1))(*blocks)
    hp = (ctypes.c_void_p * max(nb, 1))(*[(h.data_ptr() if h is not None else None) for h in Hmu])
    ld = (ctypes.c_int64 * max(nb, 1))(*[(h.stride(0) if h is not None else 0) for h in Hmu])
    check(lib.bse_project_seed(plan, nb, arr, hp, ld, _stream(stream)))


def bse_seed_free(plan):
    check(lib.bse_seed_free(plan))


def bse_project_blocks(problem, H, B, blocks, Hmu, Bmu, stream=None):
    """blocks: list of _lib.Block; Hmu / Bmu: lists of tensors or None."""
    nb = len(blocks)
    arr = (_lib.Block * max(nb, 1))(*blocks)
    hp = (ctypes.c_void_p * max(nb, 1))(*[(h.data_ptr() if h is not None else None) for h in Hmu])
    ld = (ctypes.c_int64 * max(nb, 1))(*[(h.stride(0) if h is not None else 0) for h in Hmu])
    bp = (ctypes.c_void_p * max(nb, 1))(*[(b.data_ptr() if b is not None else None) for b in Bmu])
    h_fp64 = 1 if (H is not None and H.dtype.itemsize == 16) else 0
    check(lib.bse_project_blocks(ctypes.byref(problem), _ptr(H), H.stride(0) if H is not None else 0,
                                 h_fp64, _ptr(B), nb, arr, hp, ld, bp, _stream(stream)))


def bse_dipole_weights(problem, B, blocks, weights, active, stream=None):
    """|U_mu^T B|^2 of every block into weights (device double[nblk]) and the
    index of the dipole-active block into active (device int32[1], -1: none)."""
    nb = len(blocks)
    arr = (_lib.Block * nb)(*blocks)
    check(lib.bse_dipole_weights(ctypes.byref(problem), _ptr(B), nb, arr, _ptr(weights),
                                 _ptr(active), _stream(stream)))


def bse_block_eigh_ws(n, h_fp64, prec, nrefine=0):
    return lib.bse_block_eigh_ws(n, h_fp64, prec, nrefine)


def bse_block_eigh_set_two_stage(nmin):
    """Switch point of the two-stage reduction (nmin < 0: query); returns the previous."""
    return lib.bse_block_eigh_set_two_stage(nmin)


def bse_block_eigh(Hmu, Bmu, prec, omega, pole, osc, ws, nrefine=0, stream=None):
    n = Hmu.shape[0]
    h_fp64 = 1 if Hmu.dtype.itemsize == 16 else 0
    nbytes = ws.numel() * ws.element_size()
    check(lib.bse_block_eigh(n, _ptr(Hmu), Hmu.stride(0), h_fp64, _ptr(Bmu), prec, nrefine,
                             _ptr(omega), _ptr(pole), _ptr(osc), _ptr(ws), nbytes,
                             _stream(stream)))


def bse_block_eigh_status(n, prec, nrefine, ws, stream=None, raise_on_noconv=True):
    """Counters of the last solve on ws (None: the static workspace of the
    allocation-free solver): [unrefined, non-finite, straddling clusters, 0].
    Raises BseError (BSE_ENOCONV) when eigenvalues were left unrefined or are
    not finite, unless raise_on_noconv is False."""
    st = (ctypes.c_int32 * 4)()
    rc = lib.bse_block_eigh_status(n, prec, nrefine, None if ws is None else _ptr(ws), st,
                                   _stream(stream))
    if rc != _lib.ENOCONV or raise_on_noconv:
        check(rc)
    return list(st)


def bse_sync_probe(mode, wgs, steps, buf, stream=None):
    """Microseconds per step of a lockstep chain: mode 0 one launch per step,
    mode 1 one cooperative launch with grid barriers (buf: int32[2 wgs])."""
    us = ctypes.c_double()
    check(lib.bse_sync_probe(mode, wgs, steps, _ptr(buf), ctypes.byref(us), _stream(stream)))
    return us.value


def bse_block_eigh_noalloc_max():
    return lib.bse_block_eigh_noalloc_max()


def bse_block_eigh_noalloc(Hmu, Bmu, prec, omega, pole, osc, nrefine=0, stream=None):
    """bse_block_eigh with the library's static device workspace (no allocation)."""
    n = Hmu.shape[0]
    h_fp64 = 1 if Hmu.dtype.itemsize == 16 else 0
    check(lib.bse_block_eigh_noalloc(n, _ptr(Hmu), Hmu.stride(0), h_fp64, _ptr(Bmu), prec,
                                     nrefine, _ptr(omega), _ptr(pole), _ptr(osc),
                                     _stream(stream)))


def bse_batch_eigh_ws(ns, h_fp64, prec):
    arr = (ctypes.c_int64 * len(ns))(*[int(x) for x in ns])
    return lib.bse_batch_eigh_ws(len(ns), arr, h_fp64, prec)


def bse_batch_eigh_plan(Hmus, Bmus, prec, omegas, poles, oscs, ws, stream=None):
    """Plan a lockstep solve of the blocks Hmus[b] (square tensors); returns the plan id."""
    nb = len(Hmus)
    vpa = lambda ts: (ctypes.c_void_p * nb)(*[t.data_ptr() for t in ts])
    ns = (ctypes.c_int64 * nb)(*[t.shape[0] for t in Hmus])
    lds = (ctypes.c_int64 * nb)(*[t.stride(0) for t in Hmus])
    h_fp64 = 1 if Hmus[0].dtype.itemsize == 16 else 0
    plan = ctypes.c_int64()
    check(lib.bse_batch_eigh_plan(nb, ns, vpa(Hmus), lds, h_fp64, vpa(Bmus), prec, vpa(omegas),
                                  vpa(poles), vpa(oscs), _ptr(ws),
                                  ws.numel() * ws.element_size(), ctypes.byref(plan),
                                  _stream(stream)))
    return plan.value


def bse_batch_eigh_run(plan, stream=None):
    check(lib.bse_batch_eigh_run(plan, _stream(stream)))


def bse_batch_eigh_tune(plan, stream=None):
    """Autotune the plan; returns (waves per HEMV row, trailing-update tile edge)."""
    w, t = ctypes.c_int32(), ctypes.c_int32()
    check(lib.bse_batch_eigh_tune(plan, _stream(stream), ctypes.byref(w), ctypes.byref(t)))
    return w.value, t.value


def bse_batch_eigh_config(plan, wpr, tile, stream=None):
    check(lib.bse_batch_eigh_config(plan, wpr, tile, _stream(stream)))


def bse_batch_eigh_free(plan):
    check(lib.bse_batch_eigh_free(plan))


def bse_spectrum(pole, osc, pref, eta, w, eps2, stream=None):
    check(lib.bse_spectrum(pole.numel(), _ptr(pole), _ptr(osc), float(pref), float(eta),
                           w.numel(), _ptr(w), _ptr(eps2), _stream(stream)))


def bse_haydock_ws(n):
    return int(lib.bse_haydock_ws(int(n)))


def bse_haydock(Hmu, Bmu, K, a, b, ws, stream=None):
    """K Lanczos-Haydock steps on the block: a[K], b[K+1] (b[0] = |B_mu|)."""
    import torch
    n = Hmu.shape[0]
    h64 = 1 if Hmu.dtype == torch.complex128 else 0
    check(lib.bse_haydock(n, _ptr(Hmu), Hmu.stride(0), h64, _ptr(Bmu), int(K), _ptr(a), _ptr(b),
                          _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def bse_haydock_spectrum(K, a, b, pref, eta, w, eps2, stream=None):
    check(lib.bse_haydock_spectrum(int(K), _ptr(a), _ptr(b), float(pref), float(eta), w.numel(),
                                   _ptr(w), _ptr(eps2), _stream(stream)))


def bse_eels_ws(n):
    return int(lib.bse_eels_ws(int(n)))


def bse_eels(pole, osc, c, xpole, xosc, ws, stream=None):
    """Longitudinal poles and strengths (roots of the secular equation) from
    the optical poles of bse_block_eigh; unused tail entries are (0, 0)."""
    check(lib.bse_eels(pole.numel(), _ptr(pole), _ptr(osc), float(c), _ptr(xpole), _ptr(xosc),
                       _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


# --------------------------------------------------------------------------
# kernel timing
# --------------------------------------------------------------------------
def bse_prof_enable(prefix):
    check(lib.bse_prof_enable(prefix.encode() if prefix else None))


def bse_prof_collect():
    """Wait for the recorded events; returns {kernel: (total_ms, launches)}."""
    check(lib.bse_prof_collect())
    out = {}
    for i in range(check(lib.bse_prof_count())):
        name = ctypes.create_string_buffer(32)
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        check(lib.bse_prof_get(i, name, ctypes.byref(ms), ctypes.byref(cnt)))
        out[name.value.decode()] = (ms.value, cnt.value)
    return out


def bse_prof_reset():
    check(lib.bse_prof_reset())
