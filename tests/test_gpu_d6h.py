"""GPU parity of the optional passes on a layered hexagonal (D6h) system,
whose dipole-active block is the two-dimensional E1u:

* the x-partner block of E1u (half of the block): its spectrum equals the
  oracle's partner block (the E1u spectrum without the double degeneracy) and
  its eps2 equals the whole E1u block's (FP64 1e-9 eV / 1e-10 relative,
  FP32 1e-5 eV / 1e-4);
* the longitudinal excitons of the E1u block against the oracle's secular
  equation (roots 1e-9 eV, strengths 1e-9 of the total, FP64);
* Lanczos-Haydock on the E1u block with the Krylov space exhausted against
  the block's eigenpair eps2 (1e-8 relative, FP64).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import bse as OB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CFG = dict(lattice="hex", grid=(8, 8, 1), nv=2, nc=3, nmb=64, seed=61, name="hex8")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ref():
    P = OB.make_problem(CFG)
    H = OB.hamiltonian(P)
    act = OB.dipole_active(P)
    assert act == ["E1u"]
    r = OB.solve_block(P, "E1u", H)
    wx = np.linalg.eigvalsh(OB.project(H, OB.basis_matrix(P, OB.partner_basis(P, "E1u", 0))))
    grid = synth.omega_grid_from_range(r["omega"].min(), r["omega"].max())
    e2 = OB.eps2(r["cl_e"], r["cl_w"], P["nk"], synth.ETA, grid)
    return P, r, wx, grid, e2


@pytest.mark.parametrize("precname,tol,e2tol", [("FP64", 1e-9, 1e-10), ("FP32", 1e-5, 1e-4)])
def test_e1u_partner_block(ref, precname, tol, e2tol):
    import workloads
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.system import Solver
    P, r, wx, grid, e2 = ref
    S = workloads.device_system(CFG, getattr(B, precname))
    sv = Solver(S, "E1u", wgrid=grid, partner=0)
    assert 2 * sv.blk.n == r["blk"]["n"] == 2 * len(wx)
    sv.step()
    res = sv.results()
    err = np.abs(res["omega"] - wx).max()
    e2err = np.abs(res["eps2"] - e2).max() / np.abs(e2).max()
    say("E1u x-partner", precname, "n", sv.blk.n, "spectrum err", err, "eps2 rel err", e2err)
    assert err < tol and e2err < e2tol


def test_e1u_longitudinal(ref):
    import workloads
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.system import Solver
    P, r, wx, grid, e2 = ref
    xr, wr = OB.eels(r["cl_e"], r["cl_w"], P["nk"])
    S = workloads.device_system(CFG, B.FP64)
    sv = Solver(S, "E1u", wgrid=grid)
    sv.step()
    out = sv.eels()
    say("E1u longitudinal: roots", len(out["pole"]), "oracle", len(xr))
    assert len(out["pole"]) == len(xr)
    assert np.abs(out["pole"] - xr).max() <= 1e-9
    assert np.abs(out["osc"] - wr).max() <= 1e-9 * wr.sum()


def test_e1u_haydock(ref):
    import workloads
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.system import Solver
    P, r, wx, grid, e2 = ref
    S = workloads.device_system(CFG, B.FP64)
    sv = Solver(S, "E1u", wgrid=grid)
    S.build()
    sv.project()
    sv.haydock(sv.blk.n)
    torch.cuda.synchronize()
    err = np.abs(sv.hd_eps2.cpu().numpy() - e2).max() / np.abs(e2).max()
    say("E1u Haydock K = n =", sv.blk.n, "eps2 rel err", err)
    assert err < 1e-8
