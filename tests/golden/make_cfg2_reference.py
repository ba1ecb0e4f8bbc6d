"""Writes cfg2_t1u_oracle.json: the FP64 oracle's solution of the cfg2 system.

cfg2: Oh 8x8x8 k grid, Nv = Nc = 4, Nmb = 256 (N = 8192), vector dipoles, so
the dipole-active block is T1u (n = 2160).  Stored: all block eigenvalues,
the degenerate-cluster poles and oscillator strengths, the frequency grid and
eps2 on it, and sum |B|^2.  Calls only the oracle and the input generator.

    python tests/golden/make_cfg2_reference.py      (about a minute, ~4 GB RAM)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import bse as OB  # noqa: E402


def main():
    cfg = synth.config("cfg2")
    P = OB.make_problem(cfg)
    act = OB.dipole_active(P)
    assert act == ["T1u"], act
    r = OB.solve_block(P, "T1u")
    wgrid = synth.omega_grid_from_range(r["omega"].min(), r["omega"].max())
    e2 = OB.eps2(r["cl_e"], r["cl_w"], P["nk"], synth.ETA, wgrid)
    out = dict(config="cfg2", irrep="T1u", n=int(r["blk"]["n"]), nk=int(P["nk"]),
               omega=r["omega"].tolist(), cl_e=r["cl_e"].tolist(), cl_w=r["cl_w"].tolist(),
               wmin=float(wgrid[0]), wmax=float(wgrid[-1]), nw=int(len(wgrid)),
               eps2=e2.tolist(), b2=float(np.sum(np.abs(P["B"]) ** 2)))
    with open(os.path.join(HERE, "cfg2_t1u_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
