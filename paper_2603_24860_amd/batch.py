"""Batched form: every irrep block of many systems in one lockstep solve.

For each system the H build and the projection onto all of its non-empty irrep
blocks run as usual (one bse_build and one bse_project_blocks call per system).
All blocks of all systems then go to one batched eigensolver plan
(bse_batch_eigh_*), which advances every block by one Householder step per
launch; the dipole-active block of each system gives its eps2.  The whole step
can be captured once into a HIP graph and replayed.  With seed=True, systems
whose shape the seed construction supports build only the seed pieces and
project every block straight from them (no H); the others stay dense.
"""
import math

import numpy as np
import torch

from . import bse as B
from .system import CDT


class BatchSolver:
    def __init__(self, systems, eig_prec=None, wgrids=None, eta=0.05, seed=False):
        self.systems = systems
        self.eta = eta
        self.seeded = []    # systems switched to the seed construction here (plans freed by close)
        if seed:
            for s in systems:
                if B.bse_seed_ws(s.group, s.problem, s.prec) > 0:
                    s.use_seed(direct=True)
                    self.seeded.append(s)
        self.blocks = []    # (system index, irrep, DeviceBlock)
        self.Hmu, self.Bmu, self.om, self.po, self.os = [], [], [], [], []
        self.active = []    # per system: index into self.blocks of its dipole-active block
        self.per_system = []
        prec0 = systems[0].prec
        self.eig_prec = prec0 if eig_prec is None else eig_prec
        if self.eig_prec == B.BF16X3:
            self.eig_prec = B.FP32
        for si, s in enumerate(systems):
            act, _ = s.active_irrep()
            mine = []
            for nm, _, _ in B.bse_group_irreps(s.group):
                blk = s.block(nm)
                if blk.n == 0:
                    continue
                if nm == act:
                    self.active.append(len(self.blocks))
                mine.append(len(self.blocks))
                self.blocks.append((si, nm, blk))
                n = blk.n
                self.Hmu.append(torch.empty((n, n), dtype=CDT[s.prec], device=s.device))
                self.Bmu.append(torch.empty(n, dtype=torch.complex128, device=s.device))
                self.om.append(torch.empty(n, dtype=torch.float64, device=s.device))
                self.po.append(torch.empty_like(self.om[-1]))
                self.os.append(torch.empty_like(self.om[-1]))
            self.per_system.append(mine)
        h64 = 1 if self.Hmu[0].dtype == torch.complex128 else 0
        nbytes = B.bse_batch_eigh_ws([h.shape[0] for h in self.Hmu], h64, self.eig_prec)
        if nbytes == 0:
            raise B.BseError(-1, B.lib.bse_last_error().decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=systems[0].device)
        self.plan = B.bse_batch_eigh_plan(self.Hmu, self.Bmu, self.eig_prec, self.om, self.po,
                                          self.os, self.ws)
        self.wpr, self.htile = 4, 64
        self.w, self.eps2 = [], []
        for si, s in enumerate(systems):
            wg = wgrids[si] if wgrids is not None else np.linspace(-10, 20, 2000)
            self.w.append(torch.as_tensor(np.asarray(wg, dtype=np.float64), device=s.device))
            self.eps2.append(torch.empty_like(self.w[-1]))
        self.graph = None

    def build_and_project(self):
        for si, s in enumerate(self.systems):
            s.build()
            idx = self.per_system[si]
            blks = [self.blocks[i][2].c for i in idx]
            if getattr(s, "seed_direct", False):
                B.bse_project_seed(s.seed_plan, blks, [self.Hmu[i] for i in idx])
                B.bse_project_blocks(s.problem, None, s.t["B"], blks, [None] * len(idx),
                                     [self.Bmu[i] for i in idx])
            else:
                B.bse_project_blocks(s.problem, s.H, s.t["B"], blks,
                                     [self.Hmu[i] for i in idx], [self.Bmu[i] for i in idx])

    def eigh(self):
        B.bse_batch_eigh_run(self.plan)

    def spectra(self):
        for si, s in enumerate(self.systems):
            i = self.active[si]
            B.bse_spectrum(self.po[i], self.os[i], 8 * math.pi / s.nk, self.eta, self.w[si],
                           self.eps2[si])

    def step(self):
        if self.graph is not None:
            self.graph.replay()
            return
        self.build_and_project()
        self.eigh()
        self.spectra()

    def tune(self):
        """Autotune the batched eigensolver on this batch (runs it a few times).
        Tuning rewrites the plan's launch tables, which a captured graph reads
        with the grid sizes of its capture, so it must come before capture()."""
        if self.graph is not None:
            raise RuntimeError("tune() after capture(): the captured graph keeps the grid sizes "
                               "of the old tables; tune first, then capture")
        self.build_and_project()
        self.wpr, self.htile = B.bse_batch_eigh_tune(self.plan)
        return self.wpr, self.htile

    def capture(self):
        """Record one whole step (builds, projections, batched eigh, spectra)
        into a HIP graph; later step() calls replay it."""
        for s in self.systems:
            if not getattr(s, "seed_direct", False):
                s.alloc_build()
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self.build_and_project()
            self.eigh()
            self.spectra()
        self.graph = g

    def results(self, nlow=100):
        torch.cuda.synchronize()
        out = []
        for si in range(len(self.systems)):
            blocks = {self.blocks[i][1]: self.om[i].cpu().numpy() for i in self.per_system[si]}
            a = self.active[si]
            out.append(dict(blocks=blocks, active=self.blocks[a][1],
                            pole=self.po[a].cpu().numpy(), osc=self.os[a].cpu().numpy(),
                            eps2=self.eps2[si].cpu().numpy(),
                            lowest=self.om[a][:nlow].cpu().numpy()))
        return out

    def close(self):
        self.graph = None
        B.bse_batch_eigh_free(self.plan)
        for s in self.seeded:
            B.bse_seed_free(s.seed_plan)
            s.seed_plan = None
            s.seed_ws = None
            s.use_seed(False)
        self.seeded = []
