"""Writes cfg3_t1u_oracle.json: the FP64 oracle's solution of the cfg3 system.

cfg3: Oh 12x12x12 k grid (1728 k), Nv = 4, Nc = 6, Nmb = 384 (N = 41472),
vector dipoles, so the dipole-active block is T1u (n = 10080).  The full FP64
H (27.5 GB) is never held: H_mu is formed one k orbit of rows at a time by
oracle.bse.project_streamed, then diagonalised densely.  Stored: all block
eigenvalues, the degenerate-cluster poles, strengths and sizes, the frequency
grid and eps2 on it, sum |B|^2 and the stage times.  Calls only the oracle and
the input generator.

    python tests/golden/make_cfg3_reference.py            (about 30 min, ~20 GB RAM)
    python tests/golden/make_cfg3_reference.py cfg2 OUT   (the same route for cfg2)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import bse as OB  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main(name="cfg3", out=None):
    t0 = time.perf_counter()
    cfg = synth.config(name)
    P = OB.make_problem(cfg)
    t1 = time.perf_counter()
    log(f"{name}: N = {P['N']}, inputs drawn in {t1 - t0:.0f} s")
    blk = OB.isotypic_basis(P, "T1u")
    nb2 = float(np.sum(np.abs(P["B"]) ** 2))
    Bm = OB.project_vector(P, blk, P["B"])
    # the T1u block carries the whole dipole (vector dipoles, Sec. III.D.1)
    assert abs(float(np.sum(np.abs(Bm) ** 2)) - nb2) <= 1e-10 * nb2
    norb = len(blk["basis"])
    Hm = OB.project_streamed(P, blk, log=lambda o: log(
        f"  orbit {o + 1}/{norb} done, {time.perf_counter() - t1:.0f} s"))
    t2 = time.perf_counter()
    herm = float(np.abs(Hm - Hm.conj().T).max() / np.abs(Hm).max())
    log(f"H_mu (n = {blk['n']}) in {t2 - t1:.0f} s, relative anti-Hermitian part {herm:.1e}")
    del P["mv"], P["mc"]
    w, A = OB.eigh(Hm)
    t3 = time.perf_counter()
    log(f"eigh in {t3 - t2:.0f} s")
    e, s, m = OB.oscillator_strengths(w, A, Bm)
    wgrid = synth.omega_grid_from_range(w.min(), w.max())
    e2 = OB.eps2(e, s, P["nk"], synth.ETA, wgrid)
    t4 = time.perf_counter()
    res = dict(config=name, irrep="T1u", n=int(blk["n"]), nk=int(P["nk"]), N=int(P["N"]),
               omega=w.tolist(), cl_e=e.tolist(), cl_w=s.tolist(), cl_m=m.tolist(),
               wmin=float(wgrid[0]), wmax=float(wgrid[-1]), nw=int(len(wgrid)),
               eps2=e2.tolist(), b2=nb2, hmu_rel_antihermitian=herm,
               seconds=dict(inputs=t1 - t0, h_mu=t2 - t1, eigh=t3 - t2, spectrum=t4 - t3))
    out = out or os.path.join(HERE, f"{name}_t1u_oracle.json")
    with open(out, "w") as f:
        json.dump(res, f)
    log(f"wrote {out}")


if __name__ == "__main__":
    main(*sys.argv[1:])
