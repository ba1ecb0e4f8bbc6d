"""Writes cfg4_largest_oracle.json: the FP64 oracle's solution of the largest
system of the batched workload.

The batched workload (synth.batch_configs(), 64 layered D6h systems) has its
largest system at index 3: a 24x24x1 hexagonal grid, Nv = 4, Nc = 3, Nmb = 256
(N = 6912).  Stored: the full spectrum of its unsymmetrised H (the union of all
its irrep blocks must equal it), and for the dipole-active E1u block all
eigenvalues, the degenerate-cluster poles and strengths, the frequency grid and
eps2 on it.  Calls only the oracle and the input generator.

    python tests/golden/make_cfg4_reference.py      (a few minutes, ~6 GB RAM)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import bse as OB  # noqa: E402

INDEX = 3


def main():
    cfgs = synth.batch_configs()
    cfg = cfgs[INDEX]
    sizes = [c["grid"][0] * c["grid"][1] * c["grid"][2] * c["nv"] * c["nc"] for c in cfgs]
    assert sizes[INDEX] == max(sizes), sizes
    P = OB.make_problem(cfg)
    H = OB.hamiltonian(P)
    full = np.linalg.eigvalsh(H)
    act = OB.dipole_active(P)
    assert act == ["E1u"], act
    r = OB.solve_block(P, "E1u", H)
    wgrid = synth.omega_grid_from_range(r["omega"].min(), r["omega"].max())
    e2 = OB.eps2(r["cl_e"], r["cl_w"], P["nk"], synth.ETA, wgrid)
    out = dict(config=cfg["name"], index=INDEX, grid=list(cfg["grid"]), nv=cfg["nv"],
               nc=cfg["nc"], nmb=cfg["nmb"], seed=cfg["seed"], N=int(P["N"]),
               full_spectrum=full.tolist(), irrep="E1u", n=int(r["blk"]["n"]),
               nk=int(P["nk"]), omega=r["omega"].tolist(), cl_e=r["cl_e"].tolist(),
               cl_w=r["cl_w"].tolist(), wmin=float(wgrid[0]), wmax=float(wgrid[-1]),
               nw=int(len(wgrid)), eps2=e2.tolist(),
               b2=float(np.sum(np.abs(P["B"]) ** 2)))
    with open(os.path.join(HERE, "cfg4_largest_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
