"""bse_block_eigh_noalloc (static device workspace) against bse_block_eigh.

Two calls in a row on one GPU, the second with a smaller block, so the second
runs on the scratch array the first left behind: each result must equal the
allocating entry point's result on the same input (same kernels, same launch
geometry: bitwise), and both must hold the spectrum they were built with.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2603_24860_amd import bse
    return bse


def _known(n, seed, mult):
    """A = Q diag(lam) Q^dag, Q the unitary factor of a complex Gaussian matrix."""
    rng = np.random.default_rng(seed)
    nd = (n + mult - 1) // mult
    lam = np.repeat(np.sort(rng.uniform(-10, 10, nd)), mult)[:n]
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Q, _ = np.linalg.qr(X)
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    return A, b, lam


def _solve(lib, A, b, prec, h_dtype, nrefine, noalloc):
    n = A.shape[0]
    Hmu = torch.as_tensor(A, dtype=h_dtype, device="cuda")
    Bmu = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
    out = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
    if noalloc:
        lib.bse_block_eigh_noalloc(Hmu, Bmu, prec, *out, nrefine=nrefine)
    else:
        h64 = 1 if h_dtype == torch.complex128 else 0
        ws = torch.full((lib.bse_block_eigh_ws(n, h64, prec, nrefine),), 255, dtype=torch.uint8,
                        device="cuda")
        lib.bse_block_eigh(Hmu, Bmu, prec, *out, ws, nrefine=nrefine)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def test_noalloc_two_calls_match_allocating_entry(lib):
    cases = [  # (n, prec, storage, nrefine, eigenvalue bar): larger first, then smaller
        (2400, lib.FP32, torch.complex64, 0, 2e-5),
        (600, lib.FP64, torch.complex128, 100, 1e-11 * 10),
    ]
    for n, prec, hdt, K, tol in cases:
        assert lib.bse_block_eigh_ws(n, int(hdt == torch.complex128), prec, K) \
            <= lib.bse_block_eigh_noalloc_max()
    got = []
    for i, (n, prec, hdt, K, tol) in enumerate(cases):
        say("noalloc call", i + 1, "n", n, "prec", prec, "nrefine", K)
        A, b, lam = _known(n, seed=41 + i, mult=3)
        got.append((A, b, lam, _solve(lib, A, b, prec, hdt, K, noalloc=True)))
    for (n, prec, hdt, K, tol), (A, b, lam, r) in zip(cases, got):
        say("allocating entry", "n", n)
        ref = _solve(lib, A, b, prec, hdt, K, noalloc=False)
        for x, y in zip(r, ref):
            assert np.array_equal(x, y)
        err = np.abs(r[0] - np.sort(lam)).max()
        say("  eigenvalue err", err)
        assert err < tol
        assert np.isfinite(r[1]).all() and np.isfinite(r[2]).all()
        assert abs(r[2].sum() - np.sum(np.abs(b) ** 2)) <= 1e-8 * np.sum(np.abs(b) ** 2)


def test_noalloc_rejects_blocks_beyond_the_scratch(lib):
    n = 4096   # FP32 workspace 135 MB > 128 MiB
    assert lib.bse_block_eigh_ws(n, 0, lib.FP32, 0) > lib.bse_block_eigh_noalloc_max()
    Hmu = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    Bmu = torch.zeros(n, dtype=torch.complex128, device="cuda")
    out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(lib.BseError) as e:
        lib.bse_block_eigh_noalloc(Hmu, Bmu, lib.FP32, *out)
    from paper_2603_24860_amd._lib import EWORKSPACE
    assert e.value.status == EWORKSPACE
