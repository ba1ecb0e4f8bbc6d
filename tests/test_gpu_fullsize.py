"""GPU parity at the full workload sizes, in the configuration bench.py times.

* cfg2 (Oh 8x8x8, N = 8192, T1u n = 2160): the whole path (build, projection,
  block eigh, eps2) against the FP64 oracle's solution stored in
  tests/golden/cfg2_t1u_oracle.json (written by make_cfg2_reference.py from
  the oracle alone).  Lowest 100 energies within 1e-5 eV (FP32 path) /
  1e-9 eV (FP64 path) / 1e-4 eV (split-BF16 build), eps2 within 1e-4
  relative, cumulative strengths; the longitudinal excitons from the same
  eigenpairs against the oracle's secular-equation roots of the stored
  clusters (cumulative strengths, loss spectrum within 1e-4 relative).
* cfg2 and cfg3 (Oh 12^3, N = 41472): H elements sampled across the matrix
  (corners, conjugated classes, k = k', the diagonal, random pairs) against
  the oracle's element-by-element definition.  FP32 tolerance 2e-6 max|H|.
* cfg3 (Oh 12^3, Nv = 4, Nc = 6, Nmb = 384, T1u n = 10080): the whole path
  against the FP64 oracle's solution in tests/golden/cfg3_t1u_oracle.json
  (written by make_cfg3_reference.py from the oracle alone, H_mu formed row
  slab by row slab): lowest 100 energies within 1e-9 eV (FP64 path), 1e-5 eV
  (FP32 path, with and without FP64 refinement), 1e-4 eV (split-BF16 build
  with FP64 refinement of the lowest 100); eps2 within 1e-4 relative;
  cumulative strengths.  Properties that hold at any size: the T1u block has
  the closed-form dimension 10080, and its oscillator strengths sum to |B|^2
  (all dipole weight lies in T1u), with |B|^2 from the oracle's own dipoles.
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import bse as OB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_t1u_oracle.json")
GOLD3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_t1u_oracle.json")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2603_24860_amd import bse as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return B


def cfg_nk(cfg):
    return int(np.prod(cfg["grid"]))


def _match_cumulative(pole, osc, ce, cw, tol, wtol):
    """Cumulative oscillator strength agrees at every point further than tol
    from all poles; every oracle pole with weight has a GPU pole within tol."""
    tot = cw.sum()
    keep = osc > 1e-14 * tot
    p, o = pole[keep], osc[keep]
    for e, w in zip(ce, cw):
        if w > 1e-8 * tot:
            assert np.abs(p - e).min() < tol, (e, np.abs(p - e).min())
    allp = np.sort(np.concatenate([p, ce]))
    gaps = allp[1:] - allp[:-1]
    xs = (0.5 * (allp[1:] + allp[:-1]))[gaps > 2 * tol]
    for x in xs:
        assert abs(o[p < x].sum() - cw[ce < x].sum()) <= wtol * tot, x
    assert abs(osc.sum() - tot) <= wtol * tot


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precname,tol,wtol,nref", [("FP32", 1e-5, 1e-3, 0),
                                                     ("FP64", 1e-9, 1e-6, 0),
                                                     ("BF16X3", 1e-4, 1e-3, 0),
                                                     ("FP32", 1e-5, 1e-3, 100),
                                                     ("BF16X3", 1e-4, 1e-3, 100)])
def test_cfg2_end_to_end(lib, precname, tol, wtol, nref):
    import workloads
    from paper_2603_24860_amd.system import Solver
    ref = json.load(open(GOLD))
    cfg = synth.config("cfg2")
    say("cfg2 e2e", precname, "nrefine", nref)
    S = workloads.device_system(cfg, getattr(lib, precname))
    act, _ = S.active_irrep()
    assert act == ref["irrep"]
    wgrid = np.linspace(ref["wmin"], ref["wmax"], ref["nw"])
    sv = Solver(S, act, wgrid=wgrid, nrefine=nref)
    assert sv.blk.n == ref["n"]
    sv.step()
    res = sv.results()
    lowest = np.asarray(ref["omega"][:100])
    err = np.abs(res["lowest"] - lowest).max()
    say("  lowest-100 max err (eV)", err)
    assert err < tol
    e2 = np.asarray(ref["eps2"])
    e2err = np.abs(res["eps2"] - e2).max() / np.abs(e2).max()
    say("  eps2 rel err", e2err)
    assert e2err <= 1e-4
    _match_cumulative(res["pole"], res["osc"], np.asarray(ref["cl_e"]), np.asarray(ref["cl_w"]),
                      100 * tol, wtol)
    if nref == 0:
        # longitudinal excitons from the same eigenpairs (secular equation)
        xr, wr = OB.eels(np.asarray(ref["cl_e"]), np.asarray(ref["cl_w"]), cfg_nk(cfg))
        out = sv.eels()
        loss = OB.eps2(xr, wr, cfg_nk(cfg), synth.ETA, wgrid)
        lerr = np.abs(out["spectrum"] - loss).max() / np.abs(loss).max()
        say("  eels roots", len(out["pole"]), "oracle", len(xr), "loss rel err", lerr)
        _match_cumulative(out["pole"], out["osc"], xr, wr, 100 * tol, wtol)
        assert lerr <= 1e-4
    del sv, S
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precname,tol", [("FP32", 1e-5), ("BF16X3", 1e-4)])
def test_cfg2_partner_block(lib, precname, tol):
    """cfg2 x-partner block of T1u (n = 720): each eigenvalue is one of the
    oracle's degenerate T1u triples; eps2 equals the whole block's."""
    import workloads
    from paper_2603_24860_amd.system import Solver
    ref = json.load(open(GOLD))
    cfg = synth.config("cfg2")
    say("cfg2 partner block", precname)
    S = workloads.device_system(cfg, getattr(lib, precname))
    wgrid = np.linspace(ref["wmin"], ref["wmax"], ref["nw"])
    sv = Solver(S, "T1u", wgrid=wgrid, partner=0)
    assert sv.blk.n * 3 == ref["n"]
    sv.step()
    res = sv.results()
    om = np.asarray(ref["omega"])
    assert np.abs(om.reshape(-1, 3).max(axis=1) - om.reshape(-1, 3).min(axis=1)).max() < 1e-9
    err = np.abs(res["omega"] - om[::3]).max()
    e2 = np.asarray(ref["eps2"])
    e2err = np.abs(res["eps2"] - e2).max() / np.abs(e2).max()
    say("  spectrum max err (eV)", err, "eps2 rel err", e2err)
    assert err < tol
    assert e2err <= 1e-4
    del sv, S
    torch.cuda.empty_cache()


def _sample_pairs(P, rng, nrand):
    """(a, b) element indices: corners, the diagonal, k = k', conjugated
    classes and random pairs."""
    N, nk, per = P["N"], P["nk"], P["nv"] * P["nc"]
    ab = [(0, 0), (N - 1, N - 1), (0, N - 1), (N - 1, 0), (per - 1, per), (N // 2, N // 2 + 1)]
    ab += [(int(a), int(a)) for a in rng.integers(0, N, 8)]
    for k in rng.integers(0, nk, 6):
        ab.append((int(k) * per + int(rng.integers(per)), int(k) * per + int(rng.integers(per))))
    ab += [tuple(int(x) for x in rng.integers(0, N, 2)) for _ in range(nrand)]
    return ab


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_sampled_elements_full_size(lib, name):
    import workloads
    cfg = synth.config(name)
    say("sampled H elements", name, "FP32: generating inputs")
    S = workloads.device_system(cfg, lib.FP32)
    say("  building H, N =", S.N)
    H = S.build()
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    N, nk = S.N, S.nk
    per = S.nv * S.nc
    Pt = OB.make_problem(cfg, pairs=[0])  # tables only, to find conjugated classes
    conj_pairs = np.nonzero(Pt["T"]["pconj"])[0]
    ab = _sample_pairs(Pt, rng, 200)
    for p in rng.choice(conj_pairs, 6, replace=False):
        k, k2 = divmod(int(p), nk)
        ab.append((k * per + int(rng.integers(per)), k2 * per + int(rng.integers(per))))
    pairs = [(a // per) * nk + b // per for a, b in ab]
    say("  oracle elements for", len(ab), "samples")
    P = OB.make_problem(cfg, pairs=pairs)
    ref = np.array([OB.hamiltonian_element(P, a, b) for a, b in ab])
    flat = H.view(-1)
    ld = H.stride(0)
    idx = torch.tensor([a * ld + b for a, b in ab], dtype=torch.int64, device=H.device)
    got = flat[idx].cpu().numpy().astype(np.complex128)
    hmax = 0.0
    for r0 in range(0, N, 4096):  # max |H| without a full-size temporary
        hmax = max(hmax, float(H[r0:r0 + 4096].abs().max()))
    err = np.abs(got - ref).max()
    say("  max |dH| / max|H| =", err / hmax, " max|H| =", hmax)
    assert err <= 2e-6 * hmax
    del H, S, flat
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_cfg3_block_properties(lib):
    import workloads
    from paper_2603_24860_amd.system import Solver
    cfg = synth.config("cfg3")
    say("cfg3 T1u block properties FP32: generating inputs")
    S = workloads.device_system(cfg, lib.FP32)
    P = OB.make_problem(cfg, pairs=[0])
    dims = OB.block_dims_closed_form(P)
    act, _ = S.active_irrep()
    assert act == "T1u"
    sv = Solver(S, act, wgrid=np.linspace(-20, 20, 200))
    assert sv.blk.n == dims["T1u"] == 10080
    say("  solve n =", sv.blk.n)
    sv.step()
    res = sv.results()
    b2 = float(np.sum(np.abs(P["B"]) ** 2))
    say("  sum osc / |B|^2 - 1 =", res["osc"].sum() / b2 - 1)
    assert abs(res["osc"].sum() - b2) <= 1e-6 * b2
    assert np.all(np.diff(res["omega"]) >= 0)
    del sv, S
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def cfg3_host():
    import workloads
    say("cfg3: generating inputs on the host")
    return workloads.host_inputs(synth.config("cfg3"))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precname,nref,tol,wtol", [("FP64", 0, 1e-9, 1e-6),
                                                    ("FP32", 0, 1e-5, 1e-3),
                                                    ("FP32", 100, 1e-5, 1e-3),
                                                    ("BF16X3", 100, 1e-4, 1e-3)])
def test_cfg3_end_to_end(lib, cfg3_host, precname, nref, tol, wtol):
    """cfg3 against the oracle's stored solution: the precision configuration
    (FP64, FP32, refined split-BF16) at full size."""
    from paper_2603_24860_amd.system import DeviceSystem, Solver
    ref = json.load(open(GOLD3))
    cfg = synth.config("cfg3")
    group, grid, T, inputs = cfg3_host
    say("cfg3 e2e", precname, "nrefine", nref)
    S = DeviceSystem(group, grid, cfg["nv"], cfg["nc"], cfg["nmb"], T, inputs,
                     getattr(lib, precname))
    act, _ = S.active_irrep()
    assert act == ref["irrep"]
    wgrid = np.linspace(ref["wmin"], ref["wmax"], ref["nw"])
    sv = Solver(S, act, wgrid=wgrid, nrefine=nref)
    assert sv.blk.n == ref["n"] == 10080
    sv.step()
    res = sv.results()
    err = np.abs(res["lowest"] - np.asarray(ref["omega"][:100])).max()
    e2 = np.asarray(ref["eps2"])
    e2err = np.abs(res["eps2"] - e2).max() / np.abs(e2).max()
    say("  lowest-100 max err (eV)", err, "eps2 rel err", e2err)
    assert err < tol
    assert e2err <= 1e-4
    _match_cumulative(res["pole"], res["osc"], np.asarray(ref["cl_e"]), np.asarray(ref["cl_w"]),
                      100 * tol, wtol)
    del sv, S
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_cfg2_seed_build(lib):
    """cfg2 seed construction (7140 pair-orbit contractions instead of 262144):
    the same H as the dense build, and the same solution."""
    import workloads
    from paper_2603_24860_amd.system import Solver
    ref = json.load(open(GOLD))
    cfg = synth.config("cfg2")
    say("cfg2 seed build FP32")
    S = workloads.device_system(cfg, lib.FP32)
    Hd = S.build().clone()
    S.use_seed()
    Hs = S.build()
    torch.cuda.synchronize()
    d = float((Hs - Hd).abs().max()) / float(Hd.abs().max())
    say("  seed vs dense", d)
    assert d <= 1e-6
    del Hd
    sv = Solver(S, "T1u", wgrid=np.linspace(ref["wmin"], ref["wmax"], ref["nw"]))
    sv.step()
    res = sv.results()
    err = np.abs(res["lowest"] - np.asarray(ref["omega"][:100])).max()
    say("  lowest-100 max err (eV)", err)
    assert err < 1e-5
    lib.bse_seed_free(S.seed_plan)
    del sv, S
    torch.cuda.empty_cache()
