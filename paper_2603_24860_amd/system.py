"""Device-resident BSE system and the solve sequence.

DeviceSystem uploads one system's inputs (band energies, orbit-compressed pair
vectors, W per q orbit, dipoles) and the library's integer tables to the GPU
once; solve() then runs the hot path entirely through the C ABI:
bse_build -> bse_project_blocks -> bse_block_eigh -> bse_spectrum.
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib
from . import bse as B

CDT = {B.FP64: torch.complex128, B.FP32: torch.complex64, B.BF16X3: torch.complex64}
RDT = {B.FP64: torch.float64, B.FP32: torch.float32, B.BF16X3: torch.float32}


def _dev(a, dtype=None, device="cuda"):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


class DeviceBlock:
    def __init__(self, group, grid, irrep, nv, nc, device="cuda", partner=None):
        b = B.bse_block_basis(group, grid, irrep, nv, nc, partner=partner)
        self.irrep = irrep
        self.partner = partner
        self.n = int(b["n"])
        self.host = b
        self.t = {k: _dev(v, device=device) for k, v in b.items() if k != "n"}
        self.c = _lib.Block(self.n, *[ctypes.c_void_p(self.t[f].data_ptr())
                                     for f in ("mem_off", "members", "orb_off", "orb_dim",
                                               "ub_off", "ubasis")])


class DeviceSystem:
    """One system resident on the GPU.

    inputs: dict with ev[nk,nv], ec[nk,nc], vdiag[nmb], mx[nkorb,nv,nc,nmb],
    mv[ncls,nv,nv,nmb], mc[ncls,nc,nc,nmb], w[nqorb,nmb,nmb], B[nk*nv*nc] (numpy).
    tables: output of bse.bse_tables_build for (group, grid).
    """

    def __init__(self, group, grid, nv, nc, nmb, tables, inputs, prec, device="cuda"):
        self.group, self.grid = group, tuple(grid)
        self.nv, self.nc, self.nmb, self.prec = nv, nc, nmb, prec
        self.nk = int(np.prod(grid))
        self.N = self.nk * nv * nc
        self.device = device
        self.tables = tables
        cdt, rdt = CDT[prec], RDT[prec]
        t = dict(korb=_dev(tables["korb"], device=device),
                 pidx=_dev(tables["pidx"], device=device),
                 pconj=_dev(tables["pconj"], device=device),
                 ev=_dev(inputs["ev"], torch.float64, device),
                 ec=_dev(inputs["ec"], torch.float64, device),
                 vdiag=_dev(inputs["vdiag"], torch.float64, device),
                 mx=_dev(inputs["mx"], cdt, device), mv=_dev(inputs["mv"], cdt, device),
                 mc=_dev(inputs["mc"], cdt, device), w=_dev(inputs["w"], rdt, device),
                 B=_dev(inputs["B"], torch.complex128, device))
        self.t = t
        ptr = lambda x: ctypes.c_void_p(x.data_ptr())
        self.problem = _lib.Problem(
            (ctypes.c_int32 * 3)(*self.grid), nv, nc, nmb, tables["nkorb"], tables["ncls"],
            tables["nkorb"], ptr(t["korb"]), ptr(t["korb"]), ptr(t["pidx"]), ptr(t["pconj"]),
            ptr(t["ev"]), ptr(t["ec"]), ptr(t["vdiag"]), ptr(t["mx"]), ptr(t["mv"]),
            ptr(t["mc"]), ptr(t["w"]), 1 if prec == B.FP64 else 0)
        self.blocks = {}
        self.H = None
        self.seed_direct = False
        self.ws = None

    # -- allocation -------------------------------------------------------
    def alloc_build(self, ws_bytes=None):
        if self.H is None:
            self.H = torch.empty((self.N, self.N), dtype=CDT[self.prec], device=self.device)
        want = ws_bytes or B.bse_build_ws(self.problem, self.prec)
        if want == 0:
            raise B.BseError(-1, B.lib.bse_last_error().decode())
        if self.ws is None or self.ws.numel() < want:
            self.ws = torch.empty(want, dtype=torch.uint8, device=self.device)

    def block(self, irrep, partner=None):
        key = irrep if partner is None else (irrep, partner)
        if key not in self.blocks:
            self.blocks[key] = DeviceBlock(self.group, self.grid, irrep, self.nv, self.nc,
                                           self.device, partner=partner)
        return self.blocks[key]

    # -- pieces of the path ----------------------------------------------
    def use_seed(self, on=True, direct=False):
        """Build H by the seed (symmetry-accelerated) construction from now on.
        direct: keep only the seed pieces and project blocks straight from them
        (H is never formed)."""
        if on and getattr(self, "seed_plan", None) is None:
            nbytes = B.bse_seed_ws(self.group, self.problem, self.prec)
            if nbytes == 0:
                raise B.BseError(-6, B.lib.bse_last_error().decode())
            self.seed_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.seed_plan = B.bse_seed_plan(self.group, self.problem, self.prec, self.seed_ws)
        self.seed = on
        self.seed_direct = bool(on and direct)

    def build(self):
        if getattr(self, "seed", False):
            if self.seed_direct:
                B.bse_build_seed(self.seed_plan, None)
                return None
            if self.H is None:
                self.H = torch.empty((self.N, self.N), dtype=CDT[self.prec], device=self.device)
            B.bse_build_seed(self.seed_plan, self.H)
            return self.H
        self.alloc_build()
        B.bse_build(self.problem, self.prec, self.H, self.ws)
        return self.H

    def dipole_weights(self):
        """|U_mu^T B|^2 for every irrep with a non-empty block and the
        dipole-active irrep (bse_dipole_weights; one host sync)."""
        names = [nm for nm, _, _ in B.bse_group_irreps(self.group)]
        keep = [nm for nm in names if self.block(nm).n > 0]
        w = torch.empty(len(keep), dtype=torch.float64, device=self.device)
        act = torch.empty(1, dtype=torch.int32, device=self.device)
        B.bse_dipole_weights(self.problem, self.t["B"], [self.block(nm).c for nm in keep], w, act)
        wh = w.cpu().numpy()
        a = int(act.cpu()[0])
        return dict(zip(keep, map(float, wh))), (keep[a] if a >= 0 else None)

    def active_irrep(self):
        w, act = self.dipole_weights()
        if act is None:
            raise ValueError("no irrep block carries dipole weight")
        return act, w


class Solver:
    """Reusable buffers for repeated solves of one block of one system."""

    def __init__(self, system, irrep, eig_prec=None, nrefine=0, wgrid=None, eta=0.05,
                 partner=None):
        """partner = p: solve the partner-resolved block of row p of the vector
        irrep (1/d of the isotypic block, the same optical spectrum for a
        dipole along that row's axis)."""
        self.s = system
        self.blk = system.block(irrep, partner)
        n = self.blk.n
        dev = system.device
        self.eig_prec = system.prec if eig_prec is None else eig_prec
        if self.eig_prec == B.BF16X3:
            self.eig_prec = B.FP32
        self.nrefine = nrefine
        self.Hmu = torch.empty((n, n), dtype=CDT[system.prec], device=dev)
        self.Bmu = torch.empty(n, dtype=torch.complex128, device=dev)
        h64 = 1 if self.Hmu.dtype == torch.complex128 else 0
        self.ws = torch.empty(B.bse_block_eigh_ws(n, h64, self.eig_prec, nrefine),
                              dtype=torch.uint8, device=dev)
        self.omega = torch.empty(n, dtype=torch.float64, device=dev)
        self.pole = torch.empty(n, dtype=torch.float64, device=dev)
        self.osc = torch.empty(n, dtype=torch.float64, device=dev)
        self.eta = eta
        self.set_grid(wgrid if wgrid is not None else np.linspace(-10, 20, 2000))

    def set_grid(self, wgrid):
        self.w = torch.as_tensor(np.asarray(wgrid, dtype=np.float64), device=self.s.device)
        self.eps2 = torch.empty_like(self.w)

    def project(self):
        if getattr(self.s, "seed_direct", False):
            B.bse_project_seed(self.s.seed_plan, [self.blk.c], [self.Hmu])
            B.bse_project_blocks(self.s.problem, None, self.s.t["B"], [self.blk.c], [None],
                                 [self.Bmu])
            return
        B.bse_project_blocks(self.s.problem, self.s.H, self.s.t["B"], [self.blk.c], [self.Hmu],
                             [self.Bmu])

    def eigh(self):
        B.bse_block_eigh(self.Hmu, self.Bmu, self.eig_prec, self.omega, self.pole, self.osc,
                         self.ws, nrefine=self.nrefine)

    def spectrum(self):
        B.bse_spectrum(self.pole, self.osc, 8 * math.pi / self.s.nk, self.eta, self.w, self.eps2)

    def haydock_steps(self, K):
        """Enqueue K Lanczos-Haydock steps on the projected block (coefficients
        hd_a[K], hd_b[K+1]; no diagonalisation)."""
        n = self.blk.n
        dev = self.s.device
        if getattr(self, "hd_K", None) != K:
            self.hd_a = torch.empty(K, dtype=torch.float64, device=dev)
            self.hd_b = torch.empty(K + 1, dtype=torch.float64, device=dev)
            self.hd_K = K
        if getattr(self, "hd_ws", None) is None:
            self.hd_ws = torch.empty(B.bse_haydock_ws(n), dtype=torch.uint8, device=dev)
        B.bse_haydock(self.Hmu, self.Bmu, K, self.hd_a, self.hd_b, self.hd_ws)

    def haydock_spectrum(self):
        """Enqueue the continued-fraction eps2 of the last haydock_steps on the grid."""
        if getattr(self, "hd_eps2", None) is None or self.hd_eps2.shape != self.w.shape:
            self.hd_eps2 = torch.empty_like(self.w)
        B.bse_haydock_spectrum(self.hd_K, self.hd_a, self.hd_b, 8 * math.pi / self.s.nk,
                               self.eta, self.w, self.hd_eps2)

    def haydock(self, K):
        """haydock_steps(K) then haydock_spectrum()."""
        self.haydock_steps(K)
        self.haydock_spectrum()

    def longitudinal(self):
        """Enqueue the longitudinal excitons of the block (after eigh): roots of
        the secular equation with coupling 8 pi / N_k, their strengths, and
        their spectrum on the same grid and broadening as eps2."""
        n = self.blk.n
        if getattr(self, "loss", None) is None or self.loss.shape != self.w.shape:
            dev = self.s.device
            self.xpole = torch.empty(n, dtype=torch.float64, device=dev)
            self.xosc = torch.empty_like(self.xpole)
            self.xws = torch.empty(B.bse_eels_ws(n), dtype=torch.uint8, device=dev)
            self.loss = torch.empty_like(self.w)
        pref = 8 * math.pi / self.s.nk
        B.bse_eels(self.pole, self.osc, pref, self.xpole, self.xosc, self.xws)
        B.bse_spectrum(self.xpole, self.xosc, pref, self.eta, self.w, self.loss)

    def eels(self):
        """longitudinal() and its results as host arrays (roots, strengths,
        spectrum)."""
        self.longitudinal()
        torch.cuda.synchronize()
        xo = self.xosc.cpu().numpy()
        m = int(np.count_nonzero(xo))
        return dict(pole=self.xpole.cpu().numpy()[:m], osc=xo[:m],
                    spectrum=self.loss.cpu().numpy())

    def step(self):
        """One pass of the hot path: build, project, block eigh, spectrum."""
        self.s.build()
        self.project()
        self.eigh()
        self.spectrum()

    def status(self):
        """Counters of the last eigensolve (bse_block_eigh_status); raises
        BseError with BSE_ENOCONV when some of the lowest nrefine eigenvalues
        were left unrefined or the results are not finite."""
        return B.bse_block_eigh_status(self.blk.n, self.eig_prec, self.nrefine, self.ws)

    def results(self, nlow=100):
        torch.cuda.synchronize()
        return dict(omega=self.omega.cpu().numpy(), pole=self.pole.cpu().numpy(),
                    osc=self.osc.cpu().numpy(), eps2=self.eps2.cpu().numpy(),
                    lowest=self.omega[:nlow].cpu().numpy())
