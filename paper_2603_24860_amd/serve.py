"""Served form: continuous batching of BSE solves on one GPU.

Requests (a resident system, a build precision) arrive over time.  The server
keeps every registered system's inputs (band energies, orbit-compressed pair
vectors, W per q orbit, dipoles, block bases) resident in HBM and runs each
admitted request's whole path -- bse_build, bse_project_blocks (the
dipole-active block), bse_block_eigh, bse_spectrum, and the copy of the results
to pinned host memory -- on one of `slots` HIP streams, so requests that are
admitted while others run overlap on the device.  A request is admitted when a
slot is free, its HBM footprint (H, H_mu, workspaces, outputs) fits into the
budget left by the requests in flight and, for a large request, the quota of
large requests in flight is not used up; waiting requests are considered in
arrival order and one that cannot start lets later ones pass.  Requests larger
than the whole budget are rejected.  Completion is detected by a non-blocking
event query, which frees the slot and the budget.  Every request owns its buffers, so its result does not depend on
what else is in flight.
"""
import math
import time
import weakref
from collections import deque

import numpy as np
import torch

from . import bse as B
from .system import CDT

EL = {B.FP64: 16, B.FP32: 8, B.BF16X3: 8}


class Request:
    """One solve: a registered system, the build precision, the arrival time
    (seconds relative to the start of Server.run) and the number of lowest
    eigenvalues to refine in FP64 (0: none)."""
    __slots__ = ("rid", "system", "prec", "arrival", "nrefine", "start", "done", "result", "ev",
                 "bufs", "footprint", "status", "attempts", "errors")

    def __init__(self, rid, system, prec, arrival, nrefine=0):
        self.rid, self.system, self.prec, self.arrival = rid, system, prec, arrival
        self.nrefine = nrefine
        self.start = self.done = None
        self.result = None
        self.ev = None
        self.bufs = None
        self.footprint = 0
        self.status = "waiting"
        self.attempts = 0
        self.errors = []


def _free_plans(cache):
    for plan, _ in cache:
        B.bse_seed_free(plan)
    cache.clear()


class ServedSystem:
    """A registered, resident system: inputs of one precision class and its
    dipole-active block (FP64 inputs for FP64 requests, FP32 otherwise).
    seed_slots > 0: requests of the inputs' own precision use the seed
    construction without H (pieces only, block projected straight from them),
    one seed plan per stream slot so that requests in flight do not share
    pieces; split-BF16 requests, and shapes the seed construction does not
    support, keep the dense build."""

    def __init__(self, name, dev_system, wgrid, eta=0.05, seed_slots=0):
        self.name = name
        self.s = dev_system
        self.irrep, _ = dev_system.active_irrep()
        self.blk = dev_system.block(self.irrep)
        self.w = torch.as_tensor(np.asarray(wgrid, dtype=np.float64), device=dev_system.device)
        self.eta = eta
        self.plans = []
        if seed_slots and B.bse_seed_ws(dev_system.group, dev_system.problem,
                                        dev_system.prec) > 0:
            # plans are kept with the resident system and reused by later servers
            cache = dev_system.__dict__.get("_served_seed_plans")
            if cache is None:
                cache = dev_system._served_seed_plans = []
                weakref.finalize(dev_system, _free_plans, cache)
            while len(cache) < seed_slots:
                nbytes = B.bse_seed_ws(dev_system.group, dev_system.problem, dev_system.prec)
                ws = torch.empty(nbytes, dtype=torch.uint8, device=dev_system.device)
                cache.append((B.bse_seed_plan(dev_system.group, dev_system.problem,
                                              dev_system.prec, ws), ws))
            self.plans = [pl for pl, _ in cache[:seed_slots]]
            torch.cuda.synchronize(dev_system.device)  # plans are used from the serving streams

    def seeded(self, prec):
        return bool(self.plans) and prec == self.s.prec

    def footprint(self, prec, nrefine=0):
        s, n = self.s, self.blk.n
        el = EL[prec]
        eig_prec = B.FP32 if prec == B.BF16X3 else prec
        h64 = 1 if prec == B.FP64 else 0
        build = 0 if self.seeded(prec) else s.N * s.N * el + B.bse_build_ws(s.problem, prec)
        return (build + n * n * el + 16 * n
                + B.bse_block_eigh_ws(n, h64, eig_prec, nrefine) + 3 * 8 * n + 8 * self.w.numel())


class Server:
    """slots: HIP streams (requests in flight); hbm_budget: bytes of HBM the
    requests in flight may hold together; a request whose footprint exceeds
    big_bytes is large, and at most big_slots large requests are in flight, so
    small requests are not queued behind long ones.

    A request whose launch raises (a BseError from the library, a device
    allocation failure) or whose results come back non-finite gives back its
    slot and HBM share and is queued again, up to max_retries more attempts;
    after that it is marked "failed" (Server.failed) and the others go on.
    fault(req), when set, is called before each attempt's work and may raise:
    a host-side hook that lets tests make an attempt fail."""

    def __init__(self, slots=4, hbm_budget=288e9, device="cuda", big_bytes=4e9, big_slots=1,
                 seed=False, max_retries=2):
        self.device = device
        self.max_retries = max_retries
        self.fault = None
        self.failed = []
        self.seed = seed
        self.nslots = slots
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.free = list(range(slots))
        self.budget = float(hbm_budget)
        self.big_bytes = float(big_bytes)
        self.big_slots = big_slots
        self.big_inflight = 0
        self.max_big = 0
        self.used = 0.0
        self.max_used = 0.0
        self.systems = {}
        self.waiting = deque()
        self.running = {}
        self.finished = []
        self.rejected = []

    def register(self, name, dev_system, wgrid):
        self.systems[name] = ServedSystem(name, dev_system, wgrid,
                                          seed_slots=self.nslots if self.seed else 0)

    # -- one request's path on its stream ----------------------------------
    def _launch(self, req, slot):
        ss = self.systems[req.system]
        s = ss.s
        st = self.streams[slot]
        prec = req.prec
        eig_prec = B.FP32 if prec == B.BF16X3 else prec
        n = ss.blk.n
        h = st.cuda_stream
        if self.fault is not None:
            self.fault(req)
        with torch.cuda.stream(st):
            Hmu = torch.empty((n, n), dtype=CDT[prec], device=self.device)
            Bmu = torch.empty(n, dtype=torch.complex128, device=self.device)
            if ss.seeded(prec):  # seed pieces of this slot's plan, no H
                plan = ss.plans[slot]
                B.bse_build_seed(plan, None, stream=h)
                B.bse_project_seed(plan, [ss.blk.c], [Hmu], stream=h)
                B.bse_project_blocks(s.problem, None, s.t["B"], [ss.blk.c], [None], [Bmu],
                                     stream=h)
            else:
                H = torch.empty((s.N, s.N), dtype=CDT[prec], device=self.device)
                bws = torch.empty(max(B.bse_build_ws(s.problem, prec), 256), dtype=torch.uint8,
                                  device=self.device)
                B.bse_build(s.problem, prec, H, bws, stream=h)
                B.bse_project_blocks(s.problem, H, s.t["B"], [ss.blk.c], [Hmu], [Bmu], stream=h)
                del H, bws  # freed for later work on this stream only (stream-ordered pool)
            h64 = 1 if prec == B.FP64 else 0
            ews = torch.empty(B.bse_block_eigh_ws(n, h64, eig_prec, req.nrefine),
                              dtype=torch.uint8, device=self.device)
            om = torch.empty(n, dtype=torch.float64, device=self.device)
            po, osc = torch.empty_like(om), torch.empty_like(om)
            B.bse_block_eigh(Hmu, Bmu, eig_prec, om, po, osc, ews, nrefine=req.nrefine, stream=h)
            e2 = torch.empty_like(ss.w)
            B.bse_spectrum(po, osc, 8 * math.pi / s.nk, ss.eta, ss.w, e2, stream=h)
            host = {k: torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                    for k, t in (("omega", om), ("pole", po), ("osc", osc), ("eps2", e2))}
            for k, t in (("omega", om), ("pole", po), ("osc", osc), ("eps2", e2)):
                host[k].copy_(t, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        req.bufs = (Hmu, Bmu, ews, om, po, osc, e2, host)
        req.ev = ev

    # -- scheduling --------------------------------------------------------
    def _admit(self, now):
        """Admit waiting requests in arrival order while a slot is free.  A
        request that does not fit the HBM left or the large-request quota
        waits, and later requests that do fit may pass it; a request larger
        than the whole budget is rejected."""
        i = 0
        while self.free and i < len(self.waiting):
            req = self.waiting[i]
            fp = self.systems[req.system].footprint(req.prec, req.nrefine)
            if fp > self.budget:
                del self.waiting[i]
                req.status = "rejected"
                self.rejected.append(req)
                continue
            big = fp > self.big_bytes
            if self.used + fp > self.budget or (big and self.big_inflight >= self.big_slots):
                i += 1
                continue
            del self.waiting[i]
            slot = self.free.pop()
            req.footprint = fp
            self.used += fp
            self.max_used = max(self.max_used, self.used)
            if big:
                self.big_inflight += 1
                self.max_big = max(self.max_big, self.big_inflight)
            req.start = now
            req.status = "running"
            req.attempts += 1
            try:
                self._launch(req, slot)
            except (B.BseError, torch.cuda.OutOfMemoryError) as e:
                req.bufs = req.ev = None
                self._release(req, slot)
                self._retry_or_fail(req, e)
                break  # let the requests in flight finish before the next attempt
            self.running[req.rid] = (req, slot)

    def _release(self, req, slot):
        self.used -= req.footprint
        if req.footprint > self.big_bytes:
            self.big_inflight -= 1
        req.footprint = 0
        self.free.append(slot)

    def _retry_or_fail(self, req, err):
        req.errors.append(str(err))
        if req.attempts <= self.max_retries:
            req.status = "waiting"
            self.waiting.appendleft(req)  # first in line again
        else:
            req.status = "failed"
            self.failed.append(req)

    def _poll(self):
        done = [rid for rid, (req, _) in self.running.items() if req.ev.query()]
        now = time.perf_counter()
        for rid in done:
            req, slot = self.running.pop(rid)
            host = req.bufs[-1]
            n = host["omega"].numel()
            result = {k: v.numpy().copy() for k, v in host.items()}
            req.bufs = None
            req.ev = None
            self._release(req, slot)
            if not all(np.isfinite(v).all() for v in result.values()):
                self._retry_or_fail(req, "non-finite results")
                continue
            req.result = result
            req.result["lowest"] = req.result["omega"][:min(100, n)]
            req.done = now
            req.status = "done"
            self.finished.append(req)
        return len(done)

    def run(self, requests, t0=None):
        """Serve `requests` (sorted by arrival, seconds relative to t0); returns
        the finished ones when every request is finished, rejected or failed."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter() if t0 is None else t0
        for r in pending:
            r.arrival += t0
        while pending or self.waiting or self.running:
            now = time.perf_counter()
            while pending and pending[0].arrival <= now:
                self.waiting.append(pending.popleft())
            self._poll()
            self._admit(time.perf_counter())
            if not self._poll() and pending and not self.waiting and not self.running:
                time.sleep(max(0.0, min(0.001, pending[0].arrival - time.perf_counter())))
        return self.finished

    @staticmethod
    def latency_stats(reqs):
        lat = np.array([r.done - r.arrival for r in reqs])
        return dict(p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3), count=int(len(lat)))
