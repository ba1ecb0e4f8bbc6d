"""GPU parity of the longitudinal excitons (secular equation, Sec. III.D.2)
through the C ABI, against the oracle's bisection.

* Kernel on synthetic poles (ascending, a third of them dark, some below the
  1e-14 relative cut; strengths uniform, spread over eight decades, or mostly
  1e-9 weak): the same number of roots, roots within 1e-11 eV,
  strengths within 1e-10 of the total; unused tail entries are (0, 0).
* Closed forms: one weighted pole p with strength w has the single root
  p + c w with strength w; no weighted pole gives no root.
* cfg1 end to end (FP64, FP32): the longitudinal poles from the GPU block
  eigenpairs against the oracle's from its own eigenpairs (FP64: roots within
  1e-9 eV; FP32: every oracle root with weight has a GPU root within 1e-3 eV
  and cumulative strengths agree), and the loss spectrum within 1e-4 relative.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import bse as OB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2603_24860_amd import bse as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return B


def _gpu_eels(lib, pole, osc, c):
    n = len(pole)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")
    xp = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    xo = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.empty(lib.bse_eels_ws(n), dtype=torch.uint8, device="cuda")
    lib.bse_eels(t(pole), t(osc), c, xp, xo, ws)
    torch.cuda.synchronize()
    return xp.cpu().numpy(), xo.cpu().numpy()


@pytest.mark.parametrize("kind", ["uniform", "skewed", "mostly_weak"])
def test_eels_kernel_against_oracle(lib, kind):
    rng = np.random.default_rng(21)
    n = 777
    pole = np.sort(rng.uniform(0.5, 15.0, n))
    osc = rng.uniform(0, 1, n)
    if kind == "skewed":
        osc = osc ** 8  # strengths over eight decades
    elif kind == "mostly_weak":
        osc[rng.random(n) < 0.9] *= 1e-9  # roots pressed against their poles
    osc[rng.random(n) < 0.33] = 0.0
    osc[rng.integers(0, n, 5)] = 1e-20  # below the relative cut
    nk = 64
    c = 8 * math.pi / nk
    say("eels kernel n =", n, kind)
    xr, wr = OB.eels(pole, osc, nk)
    xp, xo = _gpu_eels(lib, pole, osc, c)
    m = len(xr)
    assert np.all(xo[:m] > 0) and np.all(xp[m:] == 0) and np.all(xo[m:] == 0)
    derr = np.abs(xp[:m] - xr).max()
    werr = np.abs(xo[:m] - wr).max() / wr.sum()
    say("  roots", m, "max |dx|", derr, "max |dw|/sum w", werr)
    assert derr <= 1e-11 and werr <= 1e-10


def test_eels_closed_forms(lib):
    c = 0.3
    xp, xo = _gpu_eels(lib, [1.0, 2.0, 3.5, 4.0, 7.0], [0, 0.5, 0, 0, 0], c)
    assert abs(xp[0] - (2.0 + c * 0.5)) <= 1e-14 * 3 and abs(xo[0] - 0.5) <= 1e-13
    assert np.all(xp[1:] == 0) and np.all(xo[1:] == 0)
    xp, xo = _gpu_eels(lib, [1.0, 2.0, 3.0], [0.0, 0.0, 0.0], c)
    assert np.all(xp == 0) and np.all(xo == 0)
    xp, xo = _gpu_eels(lib, [2.5], [1.25], c)
    assert abs(xp[0] - (2.5 + c * 1.25)) <= 1e-14 * 3 and abs(xo[0] - 1.25) <= 1e-13


def _match(pole, osc, ce, cw, tol, wtol):
    """Every reference pole with weight has a GPU pole within tol; cumulative
    strengths agree between poles further apart than 2 tol."""
    tot = cw.sum()
    for e, w in zip(ce, cw):
        if w > 1e-8 * tot:
            assert np.abs(pole - e).min() < tol, (e, np.abs(pole - e).min())
    allp = np.sort(np.concatenate([pole, ce]))
    gaps = allp[1:] - allp[:-1]
    for x in (0.5 * (allp[1:] + allp[:-1]))[gaps > 2 * tol]:
        assert abs(osc[pole < x].sum() - cw[ce < x].sum()) <= wtol * tot, x
    assert abs(osc.sum() - tot) <= wtol * tot


@pytest.mark.parametrize("precname", ["FP64", "FP32"])
def test_eels_cfg1_end_to_end(lib, precname):
    import workloads
    from paper_2603_24860_amd.system import Solver
    cfg = synth.config("cfg1")
    say("eels cfg1", precname)
    P = OB.make_problem(cfg)
    act = OB.dipole_active(P)[0]
    r = OB.solve_block(P, act, OB.hamiltonian(P))
    xr, wr = OB.eels(r["cl_e"], r["cl_w"], P["nk"])
    wgrid = synth.omega_grid_from_range(r["omega"].min(), xr.max())
    S = workloads.device_system(cfg, getattr(lib, precname))
    sv = Solver(S, act, wgrid=wgrid)
    sv.step()
    out = sv.eels()
    ref = OB.eps2(xr, wr, P["nk"], synth.ETA, wgrid)
    lerr = np.abs(out["spectrum"] - ref).max() / np.abs(ref).max()
    say("  roots gpu", len(out["pole"]), "oracle", len(xr), "loss rel err", lerr,
        "lowest", out["pole"][0], xr[0])
    if precname == "FP64":
        assert len(out["pole"]) == len(xr)
        assert np.abs(out["pole"] - xr).max() <= 1e-9
        assert np.abs(out["osc"] - wr).max() <= 1e-9 * wr.sum()
    else:
        _match(out["pole"], out["osc"], xr, wr, 1e-3, 1e-3)
    assert lerr <= 1e-4
    # longitudinal poles lie strictly above the lowest weighted optical pole
    assert out["pole"][0] > r["cl_e"][r["cl_w"] > 1e-14 * r["cl_w"].sum()][0]
