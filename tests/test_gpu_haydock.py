"""GPU parity of Lanczos-Haydock (bse_haydock, bse_haydock_spectrum) through
the C ABI, against the oracle's plain Lanczos and continued fraction.

* Coefficients: the first min(K, n, 24) a_j, b_j within 1e-10 relative to
  max|H| sqrt(n) (FP64 arithmetic on both sides; FP32 storage is compared with the
  oracle run on the same FP32-rounded matrix).  Later coefficients drift apart
  as orthogonality is lost differently under different rounding, so they are
  not compared one by one.  Sizes 1 (the first residual vanishes
  up to rounding), 5, 100, 2049
  (two LDS column chunks and a ragged last workgroup) and 9000 (four rows per
  wave).
* Continued fraction kernel: eps2 within 1e-12 relative of the oracle's.
* cfg1 end to end: the Haydock eps2 of the projected T1u block equals the
  block's eigenpair eps2 (oracle) within 1e-8 (FP64) / 1e-4 (FP32) once the
  weighted Krylov space is exhausted (K = 100 > 54 weighted clusters).
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


def _herm(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return (X + X.conj().T) / 2, rng.normal(size=n) + 1j * rng.normal(size=n)


def _gpu(lib, H, b, K, dtype):
    n = H.shape[0]
    Ht = torch.as_tensor(H, dtype=dtype, device="cuda")
    Bt = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
    a = torch.full((K,), float("nan"), dtype=torch.float64, device="cuda")
    bb = torch.full((K + 1,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.empty(lib.bse_haydock_ws(n), dtype=torch.uint8, device="cuda")
    lib.bse_haydock(Ht, Bt, K, a, bb, ws)
    torch.cuda.synchronize()
    return a.cpu().numpy(), bb.cpu().numpy()


@pytest.mark.parametrize("n,K", [(1, 3), (5, 8), (100, 40), (2049, 30), (9000, 12)])
@pytest.mark.parametrize("precname", ["FP64", "FP32"])
def test_haydock_coefficients(lib, n, K, precname):
    dtype = torch.complex128 if precname == "FP64" else torch.complex64
    H, b = _herm(n, 100 + n)
    if precname == "FP32":
        H = H.astype(np.complex64).astype(np.complex128)
    say("haydock coefficients n =", n, "K =", K, precname)
    ga, gb = _gpu(lib, H, b, K, dtype)
    ra, rb = OB.haydock_coefficients(H, b, K)
    ra = np.concatenate([ra, np.zeros(K - len(ra))])
    rb = np.concatenate([rb, np.zeros(K + 1 - len(rb))])
    m = min(K, n, 24)  # past n the Krylov space is exhausted: rounding noise
    scale = np.abs(H).max() * max(1.0, math.sqrt(n))
    ea = np.abs(ga[:m] - ra[:m]).max() / scale
    eb = np.abs(gb[:m + 1] - rb[:m + 1]).max() / max(scale, rb[0])
    say("  max |da| / scale", ea, "max |db| / scale", eb)
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gb))
    assert ea < 1e-10 and eb < 1e-10
    if n == 1:  # the first residual vanishes up to rounding
        assert np.abs(gb[1:]).max() <= 1e-14 * scale


def test_haydock_spectrum_kernel(lib):
    rng = np.random.default_rng(8)
    K = 300
    a = rng.uniform(-5, 10, K)
    b = np.concatenate([[2.5], rng.uniform(0.1, 3.0, K)])
    w = np.linspace(-12, 15, 2000)
    ref = OB.haydock_eps2(a, b, 64, 0.05, w)
    t = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda")
    e2 = torch.empty(len(w), dtype=torch.float64, device="cuda")
    lib.bse_haydock_spectrum(K, t(a), t(b), 8 * math.pi / 64, 0.05, t(w), e2)
    torch.cuda.synchronize()
    err = np.abs(e2.cpu().numpy() - ref).max() / np.abs(ref).max()
    say("haydock spectrum rel err", err)
    assert err <= 1e-12


@pytest.mark.parametrize("precname,tol", [("FP64", 1e-8), ("FP32", 1e-4)])
def test_haydock_cfg1_end_to_end(lib, precname, tol):
    import workloads
    from paper_2603_24860_amd.system import Solver
    cfg = synth.config("cfg1")
    say("haydock cfg1", precname)
    P = OB.make_problem(cfg)
    r = OB.solve_block(P, "T1u", OB.hamiltonian(P))
    wgrid = synth.omega_grid_from_range(r["omega"].min(), r["omega"].max())
    ref = OB.eps2(r["cl_e"], r["cl_w"], P["nk"], synth.ETA, wgrid)
    S = workloads.device_system(cfg, getattr(lib, precname))
    sv = Solver(S, "T1u", wgrid=wgrid)
    S.build()
    sv.project()
    sv.haydock(100)
    torch.cuda.synchronize()
    got = sv.hd_eps2.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("  eps2 rel err vs the block's eigenpairs", err)
    assert err < tol
    b0 = float(sv.hd_b[0])
    assert abs(b0 ** 2 - np.sum(np.abs(r["Bmu"]) ** 2)) < 1e-9 * b0 ** 2
