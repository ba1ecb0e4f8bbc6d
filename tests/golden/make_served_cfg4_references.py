"""Writes served_cfg4_oracle.json: the FP64 oracle's dipole-active block
spectra of all 64 systems of the batched workload (synth.batch_configs()),
the resident systems of the wide served mix (bench.py --workload cfg5w).

Stored per system (keyed cfg4.<index>): its shape, the dipole-active irrep,
the block size, the lowest 100 block eigenvalues (ascending) and the range
of the frequency grid.  Calls only the oracle and the input generator.

    python tests/golden/make_served_cfg4_references.py      (about 15 minutes)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import bse as OB  # noqa: E402


def main():
    out = {}
    for i, cfg in enumerate(synth.batch_configs()):
        P = OB.make_problem(cfg)
        act = OB.dipole_active(P)
        assert len(act) == 1, (i, act)
        r = OB.solve_block(P, act[0], OB.hamiltonian(P))
        wgrid = synth.omega_grid_from_range(r["omega"].min(), r["omega"].max())
        out[cfg["name"]] = dict(grid=list(cfg["grid"]), nv=cfg["nv"], nc=cfg["nc"],
                                nmb=cfg["nmb"], seed=cfg["seed"], irrep=act[0],
                                n=int(r["blk"]["n"]), omega=r["omega"][:100].tolist(),
                                wmin=float(wgrid[0]), wmax=float(wgrid[-1]), nw=int(len(wgrid)))
        print(i, cfg["name"], act[0], r["blk"]["n"], file=sys.stderr, flush=True)
    with open(os.path.join(HERE, "served_cfg4_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
