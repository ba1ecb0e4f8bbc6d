"""Writes served_oracle.json: the FP64 oracle's block spectra of the resident
systems of the served workload that have no stored solution of their own.

The served mix (bench.py --workload cfg5 / cfg5l) keeps cfg1, cfg2, (cfg3) and
three layered D6h systems of the batched family resident: the first members of
synth.batch_configs() with 8x8x1, 13x13x1 and 20x20x1 grids.  cfg2 and cfg3 have
their own files (make_cfg2_reference.py, make_cfg3_reference.py).  Stored per
system: the dipole-active irrep, all its block eigenvalues (ascending) and the
range of the frequency grid.  Calls only the oracle and the input generator.

    python tests/golden/make_served_references.py      (about a minute)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import bse as OB  # noqa: E402


def served_systems():
    """The served workload's resident systems without a file of their own."""
    pick = {8: None, 13: None, 20: None}
    for c in synth.batch_configs():
        if c["grid"][0] in pick and pick[c["grid"][0]] is None:
            pick[c["grid"][0]] = c
    return {"cfg1": synth.config("cfg1"), "d6h-8": pick[8], "d6h-13": pick[13],
            "d6h-20": pick[20]}


def main():
    out = {}
    for name, cfg in served_systems().items():
        P = OB.make_problem(cfg)
        act = OB.dipole_active(P)
        assert len(act) == 1, (name, act)
        r = OB.solve_block(P, act[0], OB.hamiltonian(P))
        wgrid = synth.omega_grid_from_range(r["omega"].min(), r["omega"].max())
        out[name] = dict(config=cfg.get("name", name), grid=list(cfg["grid"]), nv=cfg["nv"],
                         nc=cfg["nc"], nmb=cfg["nmb"], seed=cfg["seed"], irrep=act[0],
                         n=int(r["blk"]["n"]), omega=r["omega"].tolist(),
                         wmin=float(wgrid[0]), wmax=float(wgrid[-1]), nw=int(len(wgrid)))
        print(name, act[0], r["blk"]["n"], file=sys.stderr, flush=True)
    with open(os.path.join(HERE, "served_oracle.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
