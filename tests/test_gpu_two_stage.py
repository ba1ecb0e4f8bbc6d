"""GPU parity of the two-stage block eigensolver (full -> band -> tridiagonal).

Dense Hermitian matrices of known spectrum (A = Q diag(lam) Q^dag, Q unitary,
eigenvalues with multiplicity 1 or 3 like the T1u blocks) and known optical
weights |Q^dag b|^2 are solved with the two-stage path forced on (the switch
point lowered to the test's size) and held to the same bars as the
one-stage solver: eigenvalues within 1e-11 |lam| (FP64 working storage) or
the FP32 storage bar, cumulative oscillator strength within 1e-6 and every
weighted pole within 1e-9 of the exact one (FP64).  The sizes run from the
degenerate cases (n = 2, 3: no panel, a band already tridiagonal) through a
single ragged panel (33, 34, 65), several panels with a partial last one
(100, 162, 300, 600) to blocks with hundreds of panels and a bulge chase of
thousands of launches (4500, 8400).  Workspaces start as NaN bytes, so a
read of memory that no kernel wrote shows in the result.
"""
import math
import sys

import numpy as np
import pytest

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


@pytest.fixture
def two_stage_from(lib):
    """Sets the switch point for one test and restores it afterwards."""
    old = lib.bse_block_eigh_set_two_stage(-1)
    yield lambda nmin: lib.bse_block_eigh_set_two_stage(nmin)
    lib.bse_block_eigh_set_two_stage(old)


def _random_hermitian(n, seed, mult=1, spread=10.0):
    rng = np.random.default_rng(seed)
    nd = (n + mult - 1) // mult
    lam = np.repeat(np.sort(rng.uniform(-spread, spread, nd)), mult)[:n]
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Q, _ = np.linalg.qr(X)
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    return A, b, lam, Q.conj().T @ b


def _householder_hermitian(n, seed, mult=1, spread=10.0, nref=3):
    """A = Q diag(lam) Q^dag with Q a product of nref random reflectors (a
    dense matrix of known spectrum built in O(n^2)); returns Q^dag b too."""
    rng = np.random.default_rng(seed)
    nd = (n + mult - 1) // mult
    lam = np.repeat(np.sort(rng.uniform(-spread, spread, nd)), mult)[:n]
    A = np.diag(lam).astype(np.complex128)
    us = []
    for _ in range(nref):
        u = rng.normal(size=n) + 1j * rng.normal(size=n)
        u /= np.linalg.norm(u)
        us.append(u)
        Au = A @ u
        uA = u.conj() @ A
        A = A - 2 * np.outer(u, uA) - 2 * np.outer(Au, u.conj()) + 4 * (u.conj() @ Au) * np.outer(u, u.conj())
    A = 0.5 * (A + A.conj().T)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    qb = b.copy()
    for u in reversed(us):
        qb = qb - 2 * u * (u.conj() @ qb)
    return A, b, lam, qb


def _solve(lib, A, b, prec, h_dtype):
    n = A.shape[0]
    Hmu = torch.as_tensor(A, dtype=h_dtype, device="cuda")
    Bmu = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
    h64 = 1 if h_dtype == torch.complex128 else 0
    ws = torch.full((lib.bse_block_eigh_ws(n, h64, prec),), 255, dtype=torch.uint8, device="cuda")
    om = torch.empty(n, dtype=torch.float64, device="cuda")
    po, os_ = torch.empty_like(om), torch.empty_like(om)
    lib.bse_block_eigh(Hmu, Bmu, prec, om, po, os_, ws)
    torch.cuda.synchronize()
    return om.cpu().numpy(), po.cpu().numpy(), os_.cpu().numpy()


def _check_poles(lam, qb, pole, osc, tol=1e-9, wtol=1e-6):
    """Every weighted cluster of the exact spectrum has a pole within tol, and
    the cumulative strength sum_{pole < x} osc matches at every x more than
    tol away from all poles."""
    w = np.abs(qb) ** 2
    st = OB.clusters(lam, 1e-9)
    ce = np.array([lam[st[i]] for i in range(len(st) - 1)])
    cw = np.array([w[st[i]:st[i + 1]].sum() for i in range(len(st) - 1)])
    tot = cw.sum()
    keep = osc > 1e-14 * tot
    p, o = pole[keep], osc[keep]
    for e, wt in zip(ce, cw):
        if wt > 1e-8 * tot:
            assert np.abs(p - e).min() < tol, (e, np.abs(p - e).min())
    allp = np.sort(np.concatenate([p, ce]))
    mids = 0.5 * (allp[1:] + allp[:-1])
    xs = mids[(allp[1:] - allp[:-1]) > 2 * tol]
    for x in xs:
        assert abs(o[p < x].sum() - cw[ce < x].sum()) <= wtol * tot, x
    assert abs(osc.sum() - tot) <= 1e-8 * tot


@pytest.mark.parametrize("n,mult", [(2, 1), (3, 3), (33, 1), (34, 1), (65, 1), (100, 1),
                                    (162, 3), (300, 1), (600, 3)])
def test_two_stage_known_spectrum_fp64(lib, two_stage_from, n, mult):
    say("two-stage fp64", n, mult)
    two_stage_from(2)
    A, b, lam, qb = _random_hermitian(n, seed=5 * n + mult, mult=mult)
    om, po, os_ = _solve(lib, A, b, lib.FP64, torch.complex128)
    err = np.abs(om - lam).max()
    say("  max eigenvalue error", err)
    assert err < 1e-11 * max(1, np.abs(lam).max())
    _check_poles(lam, qb, po, os_)


@pytest.mark.parametrize("n,mult", [(34, 1), (162, 3), (600, 3)])
def test_two_stage_known_spectrum_fp32(lib, two_stage_from, n, mult):
    """FP32 working storage: the eigenvalues move by ~eps32 |A| (|A| = 10)."""
    say("two-stage fp32", n, mult)
    two_stage_from(2)
    A, b, lam, qb = _random_hermitian(n, seed=7 * n + mult, mult=mult)
    om, po, os_ = _solve(lib, A, b, lib.FP32, torch.complex64)
    err = np.abs(om - lam).max()
    say("  max eigenvalue error", err)
    assert err < 2e-5


@pytest.mark.parametrize("n,precname,mult", [(4500, "FP64", 3), (4500, "FP32", 1),
                                             (8400, "FP32", 3)])
def test_two_stage_large_blocks(lib, two_stage_from, n, precname, mult):
    """Blocks above the default switch point take the two-stage path: 140 to
    262 panels, then 9000 to 16800 bulge-chasing launches.  FP32 storage:
    the same bar as the one-stage solver (1e-4 at n = 4500, scaled by
    sqrt(n / 4500))."""
    say("two-stage large", n, precname, mult)
    two_stage_from(4096)
    A, b, lam, qb = _householder_hermitian(n, seed=91 + mult, mult=mult)
    h_dtype = torch.complex128 if precname == "FP64" else torch.complex64
    om, po, os_ = _solve(lib, A, b, getattr(lib, precname), h_dtype)
    err = np.abs(om - lam).max()
    say("  max eigenvalue error", err)
    if precname == "FP64":
        assert err < 1e-11 * np.abs(lam).max()
        _check_poles(lam, qb, po, os_)
    else:
        assert err < 1e-4 * math.sqrt(n / 4500)


def test_two_stage_matches_one_stage(lib, two_stage_from):
    """The same block through both reductions (FP64): eigenvalues within
    1e-12 |lam| of each other, the same total strength."""
    n = 700
    say("two-stage vs one-stage", n)
    A, b, lam, qb = _random_hermitian(n, seed=1234, mult=3)
    two_stage_from(1 << 20)
    om1, po1, os1 = _solve(lib, A, b, lib.FP64, torch.complex128)
    two_stage_from(2)
    om2, po2, os2 = _solve(lib, A, b, lib.FP64, torch.complex128)
    assert np.abs(om1 - om2).max() < 1e-12 * np.abs(lam).max()
    assert abs(os1.sum() - os2.sum()) < 1e-10 * os1.sum()


def _solve_refined(lib, A, b, nref):
    n = A.shape[0]
    Hmu = torch.as_tensor(A, dtype=torch.complex128, device="cuda")
    Bmu = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
    ws = torch.full((lib.bse_block_eigh_ws(n, 1, lib.FP32, nref),), 255, dtype=torch.uint8,
                    device="cuda")
    om = torch.empty(n, dtype=torch.float64, device="cuda")
    po, os_ = torch.empty_like(om), torch.empty_like(om)
    lib.bse_block_eigh(Hmu, Bmu, lib.FP32, om, po, os_, ws, nrefine=nref)
    st = lib.bse_block_eigh_status(n, lib.FP32, nref, ws, raise_on_noconv=False)
    torch.cuda.synchronize()
    return om.cpu().numpy(), po.cpu().numpy(), os_.cpu().numpy(), st


@pytest.mark.parametrize("n,mult,K", [(2, 1, 2), (3, 3, 2), (34, 1, 20), (65, 1, 65),
                                       (162, 3, 100), (600, 3, 100),
                                       (4500, 1, 100), (4500, 3, 100), (10300, 1, 50)])
def test_two_stage_refinement(lib, two_stage_from, n, mult, K):
    """FP32 working storage through the two-stage reduction with FP64
    refinement of the lowest K against an FP64 H_mu: the eigenvectors of T go
    back through every bulge-chasing reflector and every stage-1 panel, and
    their Rayleigh quotients reach FP64 accuracy (the bars of the one-stage
    refinement: 1e-9 |lam| and 100x below the unrefined error); the rest of
    the spectrum and the strengths are the unrefined two-stage ones (to FP64
    rounding: the chase that keeps its reflectors is a kernel of its own, so
    the last bits of its FP64 arithmetic may differ).  4500: 140 panels and 9000 chase launches (default switch point);
    10300: above the rows whose vector fits in LDS (the chase's reflectors
    applied to x in global memory)."""
    say("two-stage refinement", n, mult, K)
    if n >= 4096:
        two_stage_from(4096)
        A, b, lam, qb = _householder_hermitian(n, seed=313 + mult, mult=mult)
    else:
        two_stage_from(2)
        A, b, lam, qb = _random_hermitian(n, seed=11 * n + mult, mult=mult)
    o0, p0, s0, _ = _solve_refined(lib, A, b, 0)
    o1, p1, s1, st = _solve_refined(lib, A, b, K)
    k = min(K, n)
    ex = np.sort(lam)
    e0 = np.abs(o0[:k] - ex[:k]).max()
    e1 = np.abs(o1[:k] - ex[:k]).max()
    say("  lowest", k, "error unrefined", e0, "refined", e1, "status", st)
    assert st[:2] == [0, 0]
    assert e1 < 1e-9 * max(1.0, np.abs(lam).max())
    assert e1 <= e0 / 100 or e0 < 1e-12
    top = max(1.0, np.abs(lam).max())
    if k < n:
        assert np.abs(o0[k:] - o1[k:]).max() <= 1e-12 * top
    # a strength shares that rounding through the contour of its cluster
    assert np.abs(s0 - s1).max() <= 1e-10 * s0.sum()
    assert abs(s0.sum() - s1.sum()) <= 1e-10 * s0.sum()


def test_switch_point_query(lib, two_stage_from):
    """bse_block_eigh_set_two_stage returns the previous value; a negative
    argument only queries; the workspace query follows the switch point."""
    two_stage_from(5000)
    assert lib.bse_block_eigh_set_two_stage(-1) == 5000
    w1 = lib.bse_block_eigh_ws(4800, 0, lib.FP32)
    two_stage_from(4800)
    w2 = lib.bse_block_eigh_ws(4800, 0, lib.FP32)
    assert w2 > w1
    # refinement follows the switch point too; its two-stage workspace also
    # keeps every reflector of both stages (the chase's alone: n (n - 1) / 2
    # entries of 16 bytes)
    wr2 = lib.bse_block_eigh_ws(4800, 0, lib.FP32, 100)
    two_stage_from(1 << 20)
    wr1 = lib.bse_block_eigh_ws(4800, 0, lib.FP32, 100)
    assert wr2 != wr1 and wr2 - w2 >= 16 * 4800 * 4799 // 2 and wr1 > w1
    assert lib.bse_block_eigh_ws(4800, 0, lib.FP32) == w1


def test_two_stage_with_concurrent_kernels(lib, two_stage_from):
    """A second stream keeps the GPU busy with matrix products while the
    two-stage solve runs on the current one, so the workgroups of one launch
    start at different times (a panel column once read the panel's top row
    from memory that the first workgroup of the same launch rewrites).
    FP64 working storage: eigenvalues within 1e-11 |lam|, poles and
    strengths as in the other FP64 cases; then the FP32 storage bar."""
    n = 4500
    say("two-stage under concurrent load", n)
    two_stage_from(4096)
    A, b, lam, qb = _householder_hermitian(n, seed=97, mult=3)
    X = torch.randn(4096, 4096, device="cuda")
    side = torch.cuda.Stream()
    for prec, h_dtype in ((lib.FP64, torch.complex128), (lib.FP32, torch.complex64)):
        Hmu = torch.as_tensor(A, dtype=h_dtype, device="cuda")
        Bmu = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
        h64 = 1 if h_dtype == torch.complex128 else 0
        ws = torch.full((lib.bse_block_eigh_ws(n, h64, prec),), 255, dtype=torch.uint8, device="cuda")
        om = torch.empty(n, dtype=torch.float64, device="cuda")
        po, os_ = torch.empty_like(om), torch.empty_like(om)
        torch.cuda.synchronize()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            Y = X
            for _ in range(200):
                Y = torch.tanh(Y @ X * 1e-3)
        lib.bse_block_eigh(Hmu, Bmu, prec, om, po, os_, ws)
        torch.cuda.synchronize()
        assert torch.isfinite(Y).all()
        om, po, os_ = om.cpu().numpy(), po.cpu().numpy(), os_.cpu().numpy()
        err = np.abs(om - lam).max()
        say("  prec", prec, "max eigenvalue error", err)
        if prec == lib.FP64:
            assert err < 1e-11 * np.abs(lam).max()
            _check_poles(lam, qb, po, os_)
        else:
            assert err < 1e-4


def test_two_stage_block_of_40000(lib):
    """The top of the block-size range the served form is specified for:
    n = 40000, FP32 working storage, built on the GPU as Q diag(lam) Q^dag
    with Q a product of three reflectors (FP64, then rounded to FP32).
    Eigenvalues within the FP32 storage bar of the large-block tests
    (1e-4 sqrt(n / 4500) eV), total oscillator strength within 1e-5 of
    |Q^dag b|^2 summed, and a weighted pole near each of ten exact
    eigenvalues spread over the spectrum.  Then with FP64 refinement of the
    lowest 100 (two-stage back-transformation at this size)."""
    n = 40000
    say("two-stage n =", n)
    rng = np.random.default_rng(40000)
    lam = np.sort(rng.uniform(-10, 10, n))
    A = torch.diag(torch.as_tensor(lam, dtype=torch.complex128, device="cuda"))
    us = []
    for _ in range(3):
        u = torch.as_tensor(rng.normal(size=n) + 1j * rng.normal(size=n), device="cuda")
        u /= torch.linalg.norm(u)
        Au = A @ u
        uA = u.conj() @ A
        g = u.conj() @ Au
        A -= 2 * torch.outer(u, uA)
        A -= 2 * torch.outer(Au, u.conj())
        A += (4 * g) * torch.outer(u, u.conj())
        us.append(u)
    Hmu = A.to(torch.complex64)
    del A
    torch.cuda.empty_cache()
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    qb = torch.as_tensor(b, device="cuda")
    for u in reversed(us):
        qb = qb - 2 * u * (u.conj() @ qb)
    w = (qb.abs() ** 2).cpu().numpy()
    Bmu = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
    ws = torch.empty(lib.bse_block_eigh_ws(n, 0, lib.FP32), dtype=torch.uint8, device="cuda")
    om = torch.empty(n, dtype=torch.float64, device="cuda")
    po, os_ = torch.empty_like(om), torch.empty_like(om)
    lib.bse_block_eigh(Hmu, Bmu, lib.FP32, om, po, os_, ws)
    torch.cuda.synchronize()
    om, po, os_ = om.cpu().numpy(), po.cpu().numpy(), os_.cpu().numpy()
    err = np.abs(om - lam).max()
    say("  max eigenvalue error", err, "total strength", os_.sum(), w.sum())
    assert err < 1e-4 * math.sqrt(n / 4500)
    assert abs(os_.sum() - w.sum()) < 1e-5 * w.sum()
    keep = os_ > 0
    for i in np.linspace(0, n - 1, 10).astype(int):
        assert np.abs(po[keep] - lam[i]).min() < 1e-3
    # the same block with FP64 refinement of the lowest 100: the chase's
    # reflectors applied to x in global memory (n above the LDS form), 1249
    # stage-1 panels; the Rayleigh quotients against the FP32 H_mu remove the
    # eigensolver's error, not the rounding of H_mu itself (about 1e-6 here).
    # The spectrum is dense (mean gap 5e-4 against the FP32 cluster tolerance
    # 1.9e-3): the weights split such chains at FP64 resolution, and the
    # refinement takes the weights' clusters, so every one of the 100 refines.
    K = 100
    del ws
    torch.cuda.empty_cache()
    ws = torch.empty(lib.bse_block_eigh_ws(n, 0, lib.FP32, K), dtype=torch.uint8, device="cuda")
    om1 = torch.empty(n, dtype=torch.float64, device="cuda")
    po1, os1 = torch.empty_like(om1), torch.empty_like(om1)
    lib.bse_block_eigh(Hmu, Bmu, lib.FP32, om1, po1, os1, ws, nrefine=K)
    st = lib.bse_block_eigh_status(n, lib.FP32, K, ws, raise_on_noconv=False)
    om1 = om1.cpu().numpy()
    e0 = np.abs(om[:K] - lam[:K]).max()
    e1 = np.abs(om1[:K] - lam[:K]).max()
    say("  refined lowest", K, "error unrefined", e0, "refined", e1, "status", st)
    assert st[:2] == [0, 0]
    assert e1 < 1e-5 and e1 < e0 / 10
