"""C ABI: the library loads, exports what include/bse.h declares, its host-side
integer tables equal the oracle's bit for bit, its per-orbit bases span the
oracle's projector ranges, and invalid arguments are rejected before any
device work.  No compute kernel is launched here (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import bse as OB, groups, orbits
from paper_2603_24860_amd import _lib, bse as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "bse.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"\b(bse_[a-z0-9_]+)\s*\(", hdr))
    assert len(declared) >= 15
    so = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared:
        assert hasattr(so, name), name
    assert declared == set(_lib.EXPORTS)


@pytest.mark.parametrize("gname,grid", [("Oh", (2, 2, 2)), ("Oh", (3, 3, 3)), ("Oh", (4, 4, 4)),
                                        ("Oh", (8, 8, 8)), ("D6h", (6, 6, 1)),
                                        ("D6h", (12, 12, 1)), ("D6h", (5, 5, 1)),
                                        ("D6h", (6, 6, 3)), ("Oh", (1, 1, 1))])
def test_tables_bit_exact(gname, grid):
    g = groups.group(gname)
    T = B.bse_tables_build(gname, grid)
    O = orbits.tables(grid, g["kmat"])
    assert np.array_equal(T["korb"], O["korb"])
    assert np.array_equal(T["korb_rep"], O["korb_reps"])
    assert np.array_equal(T["porb"], O["porb"])
    assert np.array_equal(T["porb_rep"], O["porb_reps"])
    assert np.array_equal(T["pidx"], O["pidx"])
    assert np.array_equal(T["pconj"], O["pconj"])
    assert np.array_equal(T["cls_rep"], O["class_rep"])
    assert np.array_equal(T["cls_selfswap"].astype(bool), O["class_selfswap"])
    key = lambda a: sorted(r.tobytes() for r in np.asarray(a, dtype=np.int64))
    assert key(T["kperm"]) == key(O["kperm"])


@pytest.mark.parametrize("gname", ["Oh", "D6h"])
def test_group_ops_and_characters(gname):
    kmat, rcart = B.bse_group_ops(gname)
    g = groups.group(gname)
    idx = {m.astype(np.int64).tobytes(): i for i, m in enumerate(g["kmat"])}
    perm = [idx[m.astype(np.int64).tobytes()] for m in kmat]
    assert sorted(perm) == list(range(len(kmat)))
    assert np.allclose(rcart, g["rcart"][perm])
    for (nm, d, chi), (nm2, d2, chi2) in zip(B.bse_group_irreps(gname), g["irreps"]):
        assert (nm, d) == (nm2, d2) and np.array_equal(chi, chi2[perm])


@pytest.mark.parametrize("cfg", [dict(lattice="cubic", grid=(4, 4, 4), nv=3, nc=3),
                                 dict(lattice="cubic", grid=(3, 3, 3), nv=2, nc=1),
                                 dict(lattice="hex", grid=(6, 6, 1), nv=2, nc=2)])
def test_block_basis_matches_projector(cfg):
    c = dict(cfg, nmb=4, seed=1, name="t")
    P = OB.make_problem(c)
    gname = "Oh" if cfg["lattice"] == "cubic" else "D6h"
    nb = cfg["nv"] * cfg["nc"]
    for nm, d, chi in P["group"]["irreps"]:
        b = B.bse_block_basis(gname, cfg["grid"], nm, cfg["nv"], cfg["nc"])
        ob = OB.isotypic_basis(P, nm)
        assert b["n"] == ob["n"]
        assert np.array_equal(b["orb_dim"], ob["orb_dim"])
        assert np.array_equal(b["orb_off"], ob["orb_off"])
        if b["n"] == 0:
            continue
        # U assembled from the library's per-orbit coefficients
        U = np.zeros((P["N"], b["n"]))
        for o in range(len(b["orb_dim"])):
            mem = b["members"][b["mem_off"][o]:b["mem_off"][o + 1]]
            r = b["orb_dim"][o]
            Uo = b["ubasis"][b["ub_off"][o]:b["ub_off"][o + 1]].reshape(len(mem), r)
            for j in range(r):
                for i, k in enumerate(mem):
                    U[k * nb + np.arange(nb), b["orb_off"][o] + j * nb + np.arange(nb)] = Uo[i, j]
        Pm = OB.full_projector(P, nm)
        assert np.abs(U.T @ U - np.eye(b["n"])).max() < 1e-13
        assert np.abs(Pm @ U - U).max() < 1e-13


def test_invalid_arguments_rejected_on_host():
    assert B.lib.bse_group_order(7) == _lib.EINVAL
    with pytest.raises(B.BseError):
        B.bse_tables_build("Oh", (4, 4, 3))  # grid not invariant under Oh
    with pytest.raises(B.BseError):
        B.bse_block_basis("Oh", (2, 2, 2), 99, 1, 1)
    p = _lib.Problem()
    assert B.lib.bse_build(ctypes.byref(p), 0, None, 0, None, 0, None) == _lib.EINVAL
    p.grid[:] = [2, 2, 2]
    p.nv, p.nc, p.nmb, p.nkorb, p.ncls, p.nqorb, p.in_fp64 = 7, 1, 4, 1, 1, 1, 1
    assert B.lib.bse_build(ctypes.byref(p), 0, None, 0, None, 0, None) == _lib.EUNSUPPORTED
    assert B.lib.bse_block_eigh(0, None, 0, 1, None, 0, 0, None, None, None, None, 0,
                                None) == _lib.ESHAPE
    assert B.lib.bse_spectrum(4, None, None, 1.0, 0.05, 10, None, None, None) == _lib.EINVAL
    assert B.lib.bse_spectrum(0, None, None, 1.0, 0.05, 0, None, None, None) == _lib.OK
    assert B.lib.bse_eels(0, None, None, 1.0, None, None, None, 0, None) == _lib.ESHAPE
    assert B.lib.bse_eels(4, None, None, 1.0, None, None, None, 0, None) == _lib.EINVAL
    d = ctypes.c_void_p(16)  # never dereferenced: the call fails on the host first
    assert B.lib.bse_eels(4, d, d, 0.0, d, d, d, 1 << 20, None) == _lib.EINVAL
    assert B.lib.bse_eels(4, d, d, 1.0, d, d, d, 8, None) == _lib.EWORKSPACE
    assert B.lib.bse_eels_ws(0) == 0 and B.lib.bse_eels_ws(10) == 8 * 22
    # projection from seed pieces: an unknown plan is rejected before any launch
    assert B.lib.bse_project_seed(123456, 0, None, None, None, None) == _lib.EINVAL
    assert B.lib.bse_build_seed(123456, None, 0, None) == _lib.EINVAL
    assert "NULL" in B.lib.bse_last_error().decode() or B.lib.bse_last_error() is not None


def test_workload_inputs_identical_to_oracle_inputs():
    """GPU-side inputs come from the library's tables, the oracle's from its
    own; both key the same generator, so the arrays must be identical."""
    import workloads
    cfg = synth.config("cfg1")
    _, _, T, inp = workloads.host_inputs(cfg)
    P = OB.make_problem(cfg)
    for k in ("ev", "ec", "vdiag", "mx", "mv", "mc", "w"):
        assert np.array_equal(inp[k], P[k]), k
    assert np.allclose(inp["B"], P["B"], atol=1e-15)


def test_batch_eigh_validation():
    """The batched eigensolver's size checks run on the host before any device work."""
    import ctypes
    from paper_2603_24860_amd import _lib
    L = _lib.lib
    ns = (ctypes.c_int64 * 3)(10, 20, 5)
    assert L.bse_batch_eigh_ws(3, ns, 0, _lib.FP32) > 0
    assert L.bse_batch_eigh_ws(0, ns, 0, _lib.FP32) == 0
    big = (ctypes.c_int64 * 1)(16385)
    assert L.bse_batch_eigh_ws(1, big, 0, _lib.FP32) == 0
    bad = (ctypes.c_int64 * 1)(0)
    assert L.bse_batch_eigh_ws(1, bad, 0, _lib.FP32) == 0
    # a too small workspace is refused before anything is dereferenced
    fake = (ctypes.c_void_p * 3)(1, 1, 1)
    lds = (ctypes.c_int64 * 3)(10, 20, 5)
    plan = ctypes.c_int64()
    st = L.bse_batch_eigh_plan(3, ns, fake, lds, 0, fake, _lib.FP32, fake, fake, fake,
                               ctypes.c_void_p(1), 16, ctypes.byref(plan), None)
    assert st == _lib.EWORKSPACE
    assert L.bse_batch_eigh_run(12345, None) == _lib.EINVAL
    assert L.bse_batch_eigh_free(12345) == _lib.EINVAL


@pytest.mark.parametrize("cfg,irrep,rows", [
    (dict(lattice="cubic", grid=(4, 4, 4), nv=2, nc=1), "T1u", 3),
    (dict(lattice="cubic", grid=(3, 3, 3), nv=1, nc=2), "T1u", 3),
    (dict(lattice="hex", grid=(6, 6, 1), nv=1, nc=2), "E1u", 2),
])
def test_partner_basis_matches_projector(cfg, irrep, rows):
    """The library's partner-resolved basis: orthonormal, inside the range of
    the oracle's P_pp, of the oracle's dimensions; a non-vector irrep is refused."""
    c = dict(cfg, nmb=4, seed=1, name="t")
    P = OB.make_problem(c)
    gname = "Oh" if cfg["lattice"] == "cubic" else "D6h"
    nb = cfg["nv"] * cfg["nc"]
    for p in range(rows):
        b = B.bse_block_basis(gname, cfg["grid"], irrep, cfg["nv"], cfg["nc"], partner=p)
        ob = OB.partner_basis(P, irrep, p)
        assert b["n"] == ob["n"]
        assert np.array_equal(b["orb_dim"], ob["orb_dim"])
        U = np.zeros((P["N"], b["n"]))
        for o in range(len(b["orb_dim"])):
            mem = b["members"][b["mem_off"][o]:b["mem_off"][o + 1]]
            r = b["orb_dim"][o]
            Uo = b["ubasis"][b["ub_off"][o]:b["ub_off"][o + 1]].reshape(len(mem), r)
            for j in range(r):
                for i, k in enumerate(mem):
                    U[k * nb + np.arange(nb), b["orb_off"][o] + j * nb + np.arange(nb)] = Uo[i, j]
        Pm = OB.full_partner_projector(P, irrep, p)
        assert np.abs(U.T @ U - np.eye(b["n"])).max() < 1e-13
        assert np.abs(Pm @ U - U).max() < 1e-13
    with pytest.raises(B.BseError):
        B.bse_block_basis(gname, cfg["grid"], "A1g", cfg["nv"], cfg["nc"], partner=0)


def test_hip_failure_maps_to_edevice():
    """A failing HIP runtime call surfaces as BSE_EDEVICE with a message
    naming the call.  On a host without a GPU the first runtime call of an
    entry point fails for real (hipGetDevice / hipEventCreate), so this runs
    where no GPU is visible; no kernel is launched."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("needs a host without a GPU")
    buf = (ctypes.c_int32 * 2)()
    us = ctypes.c_double()
    for mode, call in ((1, b"hipGetDevice"), (0, b"hipEventCreate")):
        assert B.lib.bse_sync_probe(mode, 1, 1, buf, ctypes.byref(us), None) == _lib.EDEVICE
        msg = B.lib.bse_last_error()
        assert call in msg and b"failed" in msg, msg
    # the Python binding raises it as a BseError with that status
    with pytest.raises(B.BseError) as e:
        B.check(B.lib.bse_sync_probe(1, 1, 1, buf, ctypes.byref(us), None))
    assert e.value.status == _lib.EDEVICE
