"""GPU tests of the batched (lockstep) block eigensolver, through the C ABI.

* Blocks of mixed sizes (1 .. 600, with triple degeneracies) solved as one
  batch give bitwise the same eigenvalues, poles and strengths as solving
  each block alone (same kernels, same per-block arithmetic), FP64 and FP32.
* Against known spectra: eigenvalues within 1e-11 relative (FP64).
* After the autotuner has picked its variant, results stay within the known
  spectrum tolerance.
* The whole batched solve captured in a HIP graph and replayed three times,
  with eager work and synchronisations between replays, reproduces the eager
  results bitwise on every replay.
* Every row split and trailing-update tile the autotuner may choose gives
  the known spectra.
* cfg4 at full size (64 systems, 384 blocks up to 2304): the autotuned
  lockstep solve against single-block solves of sampled blocks, and its
  largest system (24x24x1, N = 6912) against the FP64 oracle's stored
  solution (tests/golden/cfg4_largest_oracle.json, written by
  make_cfg4_reference.py from the oracle alone): the union of its six block
  spectra equals the spectrum of the full H, the E1u block's lowest 100
  energies within 1e-5 eV and eps2 within 1e-4.
"""
import json
import os
import sys

import numpy as np
import pytest

from test_gpu_parity import (_cluster_weights, _householder_hermitian, _match_poles,
                             _random_hermitian)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                     "cfg4_largest_oracle.json")

SIZES = [(600, 3), (257, 1), (1, 1), (162, 3), (33, 1), (2, 1), (600, 1), (100, 1), (3, 3),
         (64, 1), (5, 1)]


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2603_24860_amd import bse as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return B


def _problems():
    return [_random_hermitian(n, seed=1000 + 7 * i + n, mult=m) for i, (n, m) in enumerate(SIZES)]


class _Batch:
    def __init__(self, lib, probs, prec, h_dtype):
        self.H = [torch.as_tensor(A, dtype=h_dtype, device="cuda") for A, _, _, _ in probs]
        self.B = [torch.as_tensor(b, dtype=torch.complex128, device="cuda") for _, b, _, _ in probs]
        self.om = [torch.empty(h.shape[0], dtype=torch.float64, device="cuda") for h in self.H]
        self.po = [torch.empty_like(o) for o in self.om]
        self.os = [torch.empty_like(o) for o in self.om]
        h64 = 1 if h_dtype == torch.complex128 else 0
        nbytes = lib.bse_batch_eigh_ws([h.shape[0] for h in self.H], h64, prec)
        assert nbytes > 0
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.plan = lib.bse_batch_eigh_plan(self.H, self.B, prec, self.om, self.po, self.os,
                                            self.ws)

    def host(self):
        torch.cuda.synchronize()
        return [(o.cpu().numpy(), p.cpu().numpy(), s.cpu().numpy())
                for o, p, s in zip(self.om, self.po, self.os)]


def _single(lib, A, b, prec, h_dtype):
    n = A.shape[0]
    Hmu = torch.as_tensor(A, dtype=h_dtype, device="cuda")
    Bmu = torch.as_tensor(b, dtype=torch.complex128, device="cuda")
    h64 = 1 if h_dtype == torch.complex128 else 0
    ws = torch.empty(lib.bse_block_eigh_ws(n, h64, prec), dtype=torch.uint8, device="cuda")
    om = torch.empty(n, dtype=torch.float64, device="cuda")
    po, os_ = torch.empty_like(om), torch.empty_like(om)
    lib.bse_block_eigh(Hmu, Bmu, prec, om, po, os_, ws)
    torch.cuda.synchronize()
    return om.cpu().numpy(), po.cpu().numpy(), os_.cpu().numpy()


@pytest.mark.parametrize("precname,h_dtype", [("FP64", torch.complex128),
                                              ("FP32", torch.complex64)])
def test_batch_equals_single(lib, precname, h_dtype):
    prec = getattr(lib, precname)
    probs = _problems()
    say("batch vs single", precname, [p[0].shape[0] for p in probs])
    bt = _Batch(lib, probs, prec, h_dtype)
    lib.bse_batch_eigh_run(bt.plan)
    got = bt.host()
    for (A, b, lam, Q), (om, po, os_) in zip(probs, got):
        so, sp, ss = _single(lib, A, b, prec, h_dtype)
        assert np.array_equal(om, so) and np.array_equal(po, sp) and np.array_equal(os_, ss), \
            A.shape[0]
        if prec == lib.FP64:
            assert np.abs(om - np.sort(lam)).max() < 1e-11 * max(1, np.abs(lam).max())
            ce, cw = _cluster_weights(lam, Q, b)
            _match_poles(po, os_, ce, cw, 1e-9)
    lib.bse_batch_eigh_free(bt.plan)


def test_batch_tuned(lib):
    probs = _problems()
    bt = _Batch(lib, probs, lib.FP64, torch.complex128)
    w, t = lib.bse_batch_eigh_tune(bt.plan)
    say("autotuned waves per row", w, "tile", t)
    assert w in (1, 2, 4) and t in (32, 64)
    lib.bse_batch_eigh_run(bt.plan)
    for (A, b, lam, Q), (om, po, os_) in zip(probs, bt.host()):
        assert np.abs(om - np.sort(lam)).max() < 1e-11 * max(1, np.abs(lam).max())
        ce, cw = _cluster_weights(lam, Q, b)
        _match_poles(po, os_, ce, cw, 1e-9)
    lib.bse_batch_eigh_free(bt.plan)


@pytest.mark.parametrize("tile", [64, 32])
@pytest.mark.parametrize("wpr", [4, 2, 1])
def test_batch_every_config(lib, wpr, tile):
    """Every row split and trailing-update tile the autotuner may pick gives
    the known spectra, including a block above the 2048 trailing rows from
    which the update runs on the lower tiles only (n = 2200, FP32 storage)."""
    probs = _problems() + [_householder_hermitian(2200, 19)]
    bt = _Batch(lib, probs, lib.FP32, torch.complex64)
    lib.bse_batch_eigh_config(bt.plan, wpr, tile)
    say("batch config", wpr, tile)
    lib.bse_batch_eigh_run(bt.plan)
    for (A, b, lam, _), (om, po, os_) in zip(probs, bt.host()):
        # FP32 storage moves the eigenvalues by ~eps32 |A| sqrt(n) (|A| = 10)
        err = np.abs(om - np.sort(lam)).max()
        assert err < 2e-5 * max(1.0, np.sqrt(len(lam) / 600)), (len(lam), err)
        b2 = float(np.sum(np.abs(b) ** 2))
        assert abs(os_.sum() - b2) <= 1e-6 * b2
    lib.bse_batch_eigh_free(bt.plan)


def test_batch_graph_replays(lib):
    probs = _problems()
    bt = _Batch(lib, probs, lib.FP32, torch.complex64)
    lib.bse_batch_eigh_run(bt.plan)  # eager reference
    ref = bt.host()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lib.bse_batch_eigh_run(bt.plan)
    for rep in range(3):
        for t in bt.om + bt.po + bt.os:
            t.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = bt.host()
        for (o1, p1, s1), (o2, p2, s2) in zip(ref, got):
            assert np.array_equal(o1, o2) and np.array_equal(p1, p2) and np.array_equal(s1, s2), rep
        say("graph replay", rep, "matches eager")
    del g
    lib.bse_batch_eigh_free(bt.plan)


BATCH = [
    dict(lattice="hex", grid=(6, 6, 1), nv=2, nc=2, nmb=128, seed=41, name="b0"),
    dict(lattice="hex", grid=(7, 7, 1), nv=2, nc=3, nmb=64, seed=42, name="b1"),
    dict(lattice="cubic", grid=(4, 4, 4), nv=3, nc=3, nmb=64, seed=43, name="b2"),
    dict(lattice="hex", grid=(8, 8, 1), nv=3, nc=2, nmb=128, seed=44, name="b3"),
]


def test_batched_form_against_oracle(lib):
    """All irrep blocks of four systems (D6h and Oh) in one batched solve:
    per system, the union of its block spectra is the full spectrum of H, the
    dipole-active block's lowest 100 energies and eps2 match the oracle."""
    _check_batched(lib, seed=False)


def test_batched_form_seed_against_oracle(lib):
    """The same with seed=True: every system builds only its seed pieces and
    projects all of its blocks straight from them (H is never formed, also not
    by the captured graph); same bars against the oracle."""
    _check_batched(lib, seed=True)


def _check_batched(lib, seed):
    import synth
    import workloads
    from oracle import bse as OB
    from paper_2603_24860_amd.batch import BatchSolver
    refs, grids = [], []
    for c in BATCH:
        P = OB.make_problem(c)
        H = OB.hamiltonian(P)
        act = OB.dipole_active(P)[0]
        r = OB.solve_block(P, act, H)
        refs.append((P, np.linalg.eigvalsh(H), act, r))
        grids.append(synth.omega_grid_from_range(r["omega"].min(), r["omega"].max()))
    systems = workloads.batch_systems(BATCH, lib.FP64)
    bs = BatchSolver(systems, wgrids=grids, seed=seed)
    say("batched form:", len(bs.blocks), "blocks from", len(systems), "systems, seed", seed)
    assert len(bs.seeded) == (len(systems) if seed else 0)
    bs.step()
    out = bs.results()
    for (P, full, act, r), res, w in zip(refs, out, grids):
        union = np.sort(np.concatenate(list(res["blocks"].values())))
        assert len(union) == len(full)
        err_u = np.abs(union - full).max()
        assert res["active"] == act
        err_l = np.abs(res["lowest"] - r["lowest"]).max()
        e2 = OB.eps2(r["cl_e"], r["cl_w"], P["nk"], synth.ETA, w)
        e2err = np.abs(res["eps2"] - e2).max() / np.abs(e2).max()
        say(" ", P["cfg"]["name"], "union err", err_u, "lowest err", err_l, "eps2", e2err)
        assert err_u < 1e-9 * max(1.0, np.abs(full).max())
        assert err_l < 1e-9
        assert e2err < 1e-4
    # the whole step as one HIP graph: every replay reproduces the eager step
    bs.capture()
    for rep in range(3):
        for t in bs.om + bs.eps2:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        bs.step()
        got = bs.results()
        for a, b in zip(out, got):
            assert np.array_equal(a["eps2"], b["eps2"])
            for nm in a["blocks"]:
                assert np.array_equal(a["blocks"][nm], b["blocks"][nm]), (rep, nm)
        say("  whole-step graph replay", rep, "matches eager")
    if seed:
        assert all(sy.H is None for sy in systems)
    bs.close()


@pytest.mark.timeout(900)
def test_cfg4_full_size_lockstep_against_single(lib):
    """cfg4 at full size (64 D6h systems, 384 blocks up to n = 2304, FP32),
    the autotuned lockstep solve as the bench times it: the largest system
    against the oracle (union of block spectra = full spectrum, E1u lowest 100
    and eps2); for the four largest
    blocks and four others, the batched eigenvalues agree with a single-block
    solve of the same H_mu (other HEMV forms, FP32 storage: within 2e-5 of
    the spectral radius) and the strengths sum to |B_mu|^2 (1e-6)."""
    import synth
    import workloads
    from paper_2603_24860_amd.batch import BatchSolver
    say("cfg4 full size: generating 64 systems")
    systems = workloads.batch_systems(synth.batch_configs(), lib.FP32)
    bs = BatchSolver(systems)
    ns = [b[2].n for b in bs.blocks]
    say("  blocks", len(ns), "n max", max(ns), "sum n", sum(ns))
    assert len(systems) == 64 and max(ns) > 2048
    # the largest system against the oracle's stored solution (its grid for eps2)
    ref = json.load(open(GOLD4))
    si = ref["index"]
    assert systems[si].N == ref["N"]
    bs.w[si] = torch.as_tensor(np.linspace(ref["wmin"], ref["wmax"], ref["nw"]), device="cuda")
    bs.eps2[si] = torch.empty_like(bs.w[si])
    wpr, tile = bs.tune()
    say("  autotuned", wpr, "waves per row, tiles of", tile)
    bs.step()
    torch.cuda.synchronize()
    r = bs.results()[si]
    union = np.sort(np.concatenate(list(r["blocks"].values())))
    full = np.asarray(ref["full_spectrum"])
    uerr = np.abs(union - full).max()
    lerr = np.abs(r["lowest"] - np.asarray(ref["omega"][:100])).max()
    e2 = np.asarray(ref["eps2"])
    e2err = np.abs(r["eps2"] - e2).max() / np.abs(e2).max()
    say("  largest system", ref["config"], "N", ref["N"], "union of block spectra vs oracle H",
        uerr, "E1u lowest-100", lerr, "eps2", e2err)
    assert r["active"] == ref["irrep"]
    assert len(union) == len(full) and uerr < 2e-5 * max(1.0, np.abs(full).max())
    assert lerr < 1e-5 and e2err <= 1e-4
    order = np.argsort(ns)[::-1]
    pick = list(order[:4]) + list(np.random.default_rng(7).choice(order[4:], 4, replace=False))
    for i in pick:
        i = int(i)
        n = ns[i]
        om_b = bs.om[i].cpu().numpy()
        os_b = bs.os[i].cpu().numpy()
        h, b = bs.Hmu[i], bs.Bmu[i]
        ws = torch.empty(lib.bse_block_eigh_ws(n, 0, lib.FP32), dtype=torch.uint8, device="cuda")
        om = torch.empty(n, dtype=torch.float64, device="cuda")
        po, os_ = torch.empty_like(om), torch.empty_like(om)
        lib.bse_block_eigh(h, b, lib.FP32, om, po, os_, ws)
        torch.cuda.synchronize()
        om_s = om.cpu().numpy()
        scale = max(1.0, np.abs(om_s).max())
        err = np.abs(om_b - om_s).max() / scale
        b2 = float((b.abs() ** 2).sum())
        say("  block", i, "n", n, "batched vs single", err, "osc sum / |B|^2 - 1", os_b.sum() / b2 - 1)
        assert err < 2e-5
        assert abs(os_b.sum() - b2) <= 1e-6 * b2
    bs.close()
    del bs, systems
    torch.cuda.empty_cache()
