#!/usr/bin/env python3
"""Benchmark of the symmetry-blocked BSE hot path on one MI355X.

One step = the whole path on one synthetic system with inputs resident in HBM:
bse_build (H = dE + 2 exchange - direct, complex MFMA) -> bse_project_blocks
(dipole-active T1u block) -> bse_block_eigh (all block eigenvalues and the
optical poles) -> bse_spectrum (eps2 on 2000 frequencies).

Default workload (the largest single-GPU configuration): Oh 12x12x12 k grid
(1728 k), Nv = 4, Nc = 6 (N = 41472), Nmb = 384, complex FP32 contractions,
T1u block of 10080; its results are checked against the FP64 oracle's stored
solution, and the refined split-BF16 form is timed against the plain FP64 GPU
form (solves/s at 0.1 meV).  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2516.6 / 3}   # dense MFMA TFLOP/s
HBM_PEAK = 8000.0                                             # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_flops(nk, nv, nc, nmb):
    """Algorithmic flops of one dense-mode build (all nk^2 pairs).

    stage 1: W(q) (real) times Mv, 4 flops per complex-real MAC: 4 nk^2 nv^2 nmb^2
    stage 2: conj(Mc) T, 8 flops per complex MAC:               8 nk^2 nv^2 nc^2 nmb
    exchange: Mx v Mx^dag over all N^2 elements:                 8 N^2 nmb
    """
    N = nk * nv * nc
    s1 = 4.0 * nk * nk * nv * nv * nmb * nmb
    s2 = 8.0 * nk * nk * nv * nv * nc * nc * nmb
    ex = 8.0 * N * N * nmb
    return s1, s2, ex


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, n_block, log_fn, eigh_n=2520):
    """The FP64 oracle timed stage by stage on the host's cores over a bounded
    sample of the workload, each stage scaled to the whole solve:
      * build: the H rows of every k of one k orbit of at most 16 points (all
        columns), scaled by N_k / |O|;
      * projection: those rows contracted into their rows of H_mu, scaled the
        same way;
      * block eigh: numpy.linalg.eigh (LAPACK zheevd, eigenvectors) of a
        Hermitian matrix of eigh_n rows, scaled by (n / eigh_n)^3;
      * spectrum: eps2 of n poles on the 2000-point grid (whole).
    Returns the oracle's build TFLOP/s (the metric's unit) with the per-stage
    seconds and the solves/s they add up to."""
    import synth
    from oracle import bse as OB
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    nk = int(np.prod(cfg["grid"]))
    # one k orbit of at most 16 points (the rows of every k cost the same),
    # its rows against every column
    P0 = OB.make_problem(cfg, pairs=[0])
    korb = P0["T"]["korb"]
    sizes = np.bincount(korb)
    o = int(np.argmax(np.where(sizes <= 16, sizes, 0)))
    members = np.nonzero(korb == o)[0]
    P = OB.make_problem(cfg, pairs=[int(k) * nk + kq for k in members for kq in range(nk)])
    blk = OB.isotypic_basis(P, "T1u")
    t0 = time.perf_counter()
    slab = OB.orbit_slab(P, members)
    t1 = time.perf_counter()
    OB.project_slab(P, blk, o, slab)
    t2 = time.perf_counter()
    del slab
    rng = np.random.default_rng(0)
    X = rng.normal(size=(eigh_n, eigh_n)) + 1j * rng.normal(size=(eigh_n, eigh_n))
    A = X + X.conj().T
    del X
    t3 = time.perf_counter()
    OB.eigh(A)
    t4 = time.perf_counter()
    del A
    poles = np.sort(rng.uniform(-5, 15, n_block))
    wts = rng.uniform(0, 1, n_block)
    wgrid = synth.omega_grid_from_range(poles[0], poles[-1])
    t5 = time.perf_counter()
    OB.eps2(poles, wts, nk, synth.ETA, wgrid)
    t6 = time.perf_counter()
    scale = nk / len(members)
    stage = {"build": (t1 - t0) * scale, "projection": (t2 - t1) * scale,
             "block_eigh": (t4 - t3) * (n_block / eigh_n) ** 3, "spectrum": t6 - t5}
    s1, s2, ex = build_flops(nk, cfg["nv"], cfg["nc"], cfg["nmb"])
    total = sum(stage.values())
    log_fn("cpu baseline: " + ", ".join(f"{k} {v:.1f} s" for k, v in stage.items())
           + f" (sampled in {t2 - t0 + t4 - t3 + t6 - t5:.1f} s)")
    return {"value": round((s1 + s2 + ex) / stage["build"] / 1e12, 4), "unit": "TFLOP/s",
            "cores": threads, "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "kind": "oracle",
            "stage_s": {k: round(v, 2) for k, v in stage.items()},
            "solve_s": round(total, 2), "solves_per_s": round(1.0 / total, 6),
            "sample": f"{cfg['name']}: H rows of the {len(members)} k of one k orbit against "
                      f"all {nk * cfg['nv'] * cfg['nc']} columns (build, {t1 - t0:.1f} s) and "
                      f"their T1u rows (projection, {t2 - t1:.1f} s), both x {scale:g}; "
                      f"numpy eigh of a {eigh_n}-row Hermitian matrix ({t4 - t3:.1f} s) "
                      f"x (n/{eigh_n})^3 for the n = {n_block} block; eps2 of {n_block} poles "
                      f"on 2000 points ({t6 - t5:.2f} s)"}


def traffic_file(workload, prec):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_k_direct_fused_{workload}_{prec}.md")


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2603_24860_amd", "csrc", f)
                  for f in ("bse_build.hip", "mfma_tile.h")]


def measured_traffic(workload, prec, seed=False):
    """HBM bytes per launch of k_direct_fused from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (copy-calibrated) for this workload and
    precision, or None when there are none, the kernel sources changed since
    the counters were taken, or the build is the seed construction (another
    kernel)."""
    import hashlib
    path = traffic_file(workload, prec)
    if seed or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("traffic_bytes_per_launch", "source_sha256"):
            vals[k] = v
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    if vals.get("source_sha256") != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


GOLDEN = {name: os.path.join(ROOT, "tests", "golden", f"{name}_t1u_oracle.json")
          for name in ("cfg2", "cfg3")}


def oracle_reference(workload):
    """The FP64 oracle's stored solution of the workload's T1u block (written
    by tests/golden/make_cfg*_reference.py from the oracle alone), or None."""
    path = GOLDEN.get(workload)
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


BARS = {"fp64": 1e-9, "fp32": 1e-5, "bf16x3": 1e-4}   # lowest-100 energies, eV
EPS2_BAR = 1e-4                                       # eps2, relative to its maximum


def accuracy(res, ref):
    """Lowest-100 error (eV) and relative eps2 error against the oracle."""
    err = float(np.abs(res["lowest"] - np.asarray(ref["omega"][:len(res["lowest"])])).max())
    e2 = np.asarray(ref["eps2"])
    return err, float(np.abs(res["eps2"] - e2).max() / np.abs(e2).max())


def bench_batched(args):
    """Batched form: all irrep blocks of 64 D6h systems, one lockstep eigensolver
    plan and the whole step (64 builds, projections, batched eigh, 64 spectra)
    replayed from one HIP graph."""
    import torch
    import synth
    import workloads
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.batch import BatchSolver
    prec = {"fp32": B.FP32, "fp64": B.FP64, "bf16x3": B.BF16X3}[args.prec]
    cfgs = synth.batch_configs()
    t0 = time.perf_counter()
    systems = workloads.batch_systems(cfgs, prec, log=log)
    bs = BatchSolver(systems, seed=args.seed)
    ns = [b[2].n for b in bs.blocks]
    log(f"setup {time.perf_counter() - t0:.1f} s; {len(systems)} systems, {len(ns)} blocks, "
        f"n in {min(ns)}..{max(ns)}, sum n = {sum(ns)}")
    wpr, tile = bs.tune()
    log(f"autotuner: {wpr} waves per row, trailing-update tiles of {tile}")
    bs.step()
    torch.cuda.synchronize()
    for si, r in enumerate(bs.results()):
        om = r["pole"]
        bs.w[si] = torch.as_tensor(synth.omega_grid_from_range(om.min(), om.max()),
                                   device=systems[si].device)
        bs.eps2[si] = torch.empty_like(bs.w[si])
    bs.capture()
    for _ in range(args.warmup):
        bs.step()
    torch.cuda.synchronize()
    # stage split of one eager step (not in the timed region)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    bs.build_and_project()
    ev[1].record()
    bs.eigh()
    ev[2].record()
    bs.spectra()
    ev[3].record()
    torch.cuda.synchronize()
    split = [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    # the same blocks, one bse_block_eigh call each (context for the lockstep gain)
    seq = []
    for i, h in enumerate(bs.Hmu):
        n = h.shape[0]
        ws = torch.empty(B.bse_block_eigh_ws(n, 0, bs.eig_prec), dtype=torch.uint8,
                         device=h.device)
        seq.append(ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i, h in enumerate(bs.Hmu):
        B.bse_block_eigh(h, bs.Bmu[i], bs.eig_prec, bs.om[i], bs.po[i], bs.os[i], seq[i])
    e1.record()
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    del seq
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bs.step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = wall * 1e3 / args.steps
    out = {
        "metric": "batched form: systems solved per second (all irrep blocks, one lockstep "
                  "eigensolver launch per Householder step, whole step replayed from a HIP graph)",
        "value": round(len(systems) / (ms * 1e-3), 3),
        "unit": "systems/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic (seeded; 64 layered D6h systems)",
        "config": {"workload": f"cfg4: {len(systems)} D6h systems n x n x 1, n in 6..24, "
                               f"Nv, Nc in 2..4, Nmb in 128..320; {len(ns)} irrep blocks, "
                               f"n {min(ns)}..{max(ns)}, sum n = {sum(ns)}"
                               + (f"; {len(bs.seeded)} systems by the seed construction, blocks "
                                  "projected from the seed pieces (no H)" if args.seed else ""),
                   "precision": args.prec},
        "stage_ms": {"builds_and_projections": round(split[0], 3),
                     "batched_block_eigh": round(split[1], 3), "spectra": round(split[2], 3)},
        "block_eigh_one_call_per_block_ms": round(seq_ms, 3),
        "lockstep_gain": round(seq_ms / split[1], 2),
        "autotuned_waves_per_row": wpr,
        "autotuned_her2k_tile": tile,
    }
    print(json.dumps(out), flush=True)
    bs.close()


def bench_served(args, large=False, wide=False):
    """Served form: a Poisson stream of BSE solve requests over a mix of
    resident systems (cubic cfg1 / cfg2 / cfg3 shapes and three layered D6h
    systems of the batched family, blocks of 162 to 10080; wide: all 64
    systems of the batched family), FP32 builds or split-BF16 builds with FP64
    refinement, continuous batching on four streams with admission by HBM
    footprint (288 GB).  Every result, and every result of the plain FP64 path
    it is compared with, is checked against the oracle's stored block spectrum
    of its system (lowest 100 within 0.1 meV)."""
    import torch
    import synth
    import workloads
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.serve import Request, Server
    rng = np.random.default_rng(5)
    d6 = synth.batch_configs()
    pick = {8: None, 13: None, 20: None}
    for c in d6:
        if c["grid"][0] in pick and pick[c["grid"][0]] is None:
            pick[c["grid"][0]] = c
    cfgs = {"cfg1": synth.config("cfg1"), "cfg2": synth.config("cfg2"),
            "d6h-8": pick[8], "d6h-13": pick[13], "d6h-20": pick[20]}
    if large:
        cfgs["cfg3"] = synth.config("cfg3")
    if wide:
        cfgs = {c["name"]: c for c in d6}
    t0 = time.perf_counter()
    sysobjs = {}
    for name, c in cfgs.items():
        for pname, prec in (("fp32", B.FP32), ("fp64", B.FP64)):
            sysobjs[f"{name}/{pname}"] = workloads.device_system(c, prec)
        log(f"  system {name} resident")
    # the oracle's stored block spectra of every resident system (tests/golden/, written from the
    # oracle alone) and their frequency grids
    grids = {}
    ref = {}
    with open(os.path.join(ROOT, "tests", "golden",
                           "served_cfg4_oracle.json" if wide else "served_oracle.json")) as f:
        served = json.load(f)
    for name in cfgs:
        g = served[name] if name in served else oracle_reference(name)
        ref[name] = np.asarray(g["omega"][:100])
        grids[name] = np.linspace(g["wmin"], g["wmax"], g["nw"])
    log(f"setup {time.perf_counter() - t0:.1f} s")
    # (system, input class, build precision, weight, FP64 refinement of the lowest K):
    # split-BF16 requests are refined
    mix = [("cfg1", "fp32", B.FP32, 0.15, 0), ("cfg1", "fp32", B.BF16X3, 0.10, 100),
           ("cfg2", "fp32", B.FP32, 0.15, 0), ("cfg2", "fp32", B.BF16X3, 0.15, 100),
           ("d6h-8", "fp32", B.FP32, 0.10, 0), ("d6h-13", "fp32", B.BF16X3, 0.15, 100),
           ("d6h-20", "fp32", B.FP32, 0.20, 0)]
    if large:  # a small share of cfg3 requests (T1u block 10080)
        mix += [("cfg3", "fp32", B.FP32, 0.02, 0), ("cfg3", "fp32", B.BF16X3, 0.02, 100)]
    if wide:  # every system of the batched family, FP32 or refined split BF16
        mix = ([(name, "fp32", B.FP32, 0.6 / len(cfgs), 0) for name in cfgs]
               + [(name, "fp32", B.BF16X3, 0.4 / len(cfgs), 100) for name in cfgs])
    wts = np.array([m[3] for m in mix])
    wts /= wts.sum()

    def server(slots, seed=args.seed):
        srv = Server(slots=slots, hbm_budget=288e9, seed=seed)
        for key, ds in sysobjs.items():
            srv.register(key, ds, grids[key.split("/")[0]])
        return srv

    def draw(count, fp64=False):
        out = []
        for i in range(count):
            name, cls, prec, _, nref = mix[int(rng.choice(len(mix), p=wts))]
            out.append(Request(i, f"{name}/fp64" if fp64 else f"{name}/{cls}",
                               B.FP64 if fp64 else prec, 0.0, 0 if fp64 else nref))
        return out

    # warm-up of every request type
    if wide:
        server(4).run([Request(i, f"{m[0]}/{m[1]}", m[2], 0.0, m[4]) for i, m in enumerate(mix)])
    else:
        server(4).run(draw(3 * len(mix)))
    # plain FP64 GPU form over the same mix, one request after the other
    nplain = 100 if large else 150
    t1 = time.perf_counter()
    pdone = server(1, seed=False).run(draw(nplain, fp64=True))
    pwall = time.perf_counter() - t1
    plain = nplain / pwall
    perr = max(float(np.abs(r.result["lowest"] - ref[r.system.split("/")[0]]).max())
               for r in pdone)
    pok = sum(1 for r in pdone if np.abs(r.result["lowest"] - ref[r.system.split("/")[0]]).max()
              <= 1e-4)
    # saturation throughput of the served form
    nsat = 200 if large else 400
    t1 = time.perf_counter()
    server(4).run(draw(nsat))
    sat = nsat / (time.perf_counter() - t1)
    # Poisson arrivals at 0.8 x saturation
    lam = 0.8 * sat
    nreq = max(400 if large else 1000, args.steps)
    reqs = draw(nreq)
    t = 0.0
    for r in reqs:
        t += rng.exponential(1.0 / lam)
        r.arrival = t
    srv = server(4)
    t1 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t1
    st = Server.latency_stats(done)
    err = {}
    for r in done:
        name = r.system.split("/")[0]
        key = {B.FP32: "fp32", B.BF16X3: "bf16x3"}[r.prec]
        err[key] = max(err.get(key, 0.0), float(np.abs(r.result["lowest"] - ref[name]).max()))
    ok = sum(1 for r in done if np.abs(r.result["lowest"] - ref[r.system.split("/")[0]]).max()
             <= 1e-4)
    out = {
        "metric": "served form: solves/s and p50/p99 latency (Poisson arrivals, continuous "
                  "batching on 4 streams, admission by HBM footprint <= 288 GB)",
        "value": round(len(done) / wall, 3), "unit": "solves/s",
        "n_gpus": 1, "steps": len(done), "warmup": 3 * len(mix),
        "ms_per_step": round(wall * 1e3 / len(done), 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32+bf16x3",
        "data": ("synthetic (seeded; the 64 resident D6h systems of the batched family)" if wide
                 else "synthetic (seeded; resident cubic cfg1/cfg2" + ("/cfg3" if large else "")
                 + " and three D6h systems)"),
        "config": {"workload": ("cfg5w: Poisson stream over all 64 D6h systems of the batched "
                                "family (6x6x1 .. 24x24x1 grids, E1u blocks of %d to %d), FP32 "
                                "builds or split-BF16 builds with FP64 refinement of the lowest "
                                "100" % (min(served[n]["n"] for n in cfgs),
                                         max(served[n]["n"] for n in cfgs)) if wide else
                                ("cfg5l" if large else "cfg5") + ": Poisson stream over cfg1 "
                               "(T1u 162), cfg2 (T1u 2160), " + ("cfg3 (T1u 10080), " if large
                                                                  else "")
                               + "D6h 8x8x1 / 13x13x1 / 20x20x1 (E1u) systems, FP32 builds or "
                               "split-BF16 builds with FP64 refinement of the lowest 100")
                               + ("; FP32 requests by the seed construction, block projected "
                                  "from the seed pieces (no H)" if args.seed else ""),
                   "requests": len(done),
                   "arrival_rate_per_s": round(lam, 3),
                   "mix": ([{"systems": len(cfgs), "fp32_weight": 0.6, "bf16x3_weight": 0.4,
                             "bf16x3_nrefine": 100}] if wide else
                           [{"system": m[0], "precision": {B.FP32: "fp32", B.BF16X3: "bf16x3"}[m[2]],
                             "weight": m[3], "nrefine": m[4]} for m in mix])},
        "latency_ms": {"p50": round(st["p50_ms"], 3), "p99": round(st["p99_ms"], 3),
                       "mean": round(st["mean_ms"], 3)},
        "saturation_solves_per_s": round(sat, 3),
        "plain_fp64_solves_per_s": round(plain, 3),
        "plain_fp64_solves_per_s_at_0.1meV": round(pok / pwall, 3),
        "plain_fp64_max_lowest100_err_meV_vs_oracle": round(perr * 1e3, 9),
        "served_over_plain_fp64": round((len(done) / wall) / plain, 3),
        "served_over_plain_fp64_at_0.1meV": round((ok / wall) / (pok / pwall), 3) if pok else None,
        "max_lowest100_err_meV_vs_oracle": {k: round(v * 1e3, 6) for k, v in err.items()},
        "solves_within_0.1meV": ok,
        "max_hbm_in_flight_GB": round(srv.max_used / 1e9, 3),
        "rejected": len(srv.rejected),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3",
                    help="cfg1 / cfg2 / cfg3: one system; cfg4: the batched form (64 D6h "
                         "systems); cfg5: the served form (Poisson request stream); cfg5w: "
                         "the served form over all 64 systems of the batched family; cfg5l: "
                         "the served form with a share of cfg3 requests")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times) and exit: "
                         "the reference for scaling HBM byte counters")
    ap.add_argument("--sync-probe", type=int, default=0, metavar="STEPS",
                    help="only time STEPS dependent steps of 256..1024 workgroups, one kernel "
                         "launch per step against one cooperative launch with grid barriers, "
                         "and exit (the design input of the batched form)")
    ap.add_argument("--copy-timed", type=int, default=0, metavar="K",
                    help="with --copy-mib: then time K more copies and report the achieved "
                         "read + write bandwidth (the practical HBM ceiling)")
    ap.add_argument("--seed", action="store_true",
                    help="build H by the seed construction (one contraction per pair orbit); "
                         "TFLOP/s then counts the contractions performed")
    ap.add_argument("--seed-direct", action="store_true",
                    help="with --seed: keep only the seed pieces and project the block straight "
                         "from them (H is never formed)")
    ap.add_argument("--partner", action="store_true",
                    help="solve the x-partner block of the dipole-active vector irrep (1/d of "
                         "the isotypic block, the same eps2) instead of the isotypic block")
    ap.add_argument("--eels", action="store_true",
                    help="also solve the secular equation for the longitudinal excitons and "
                         "their loss spectrum in every step (stage 'eels')")
    ap.add_argument("--haydock", type=int, default=0, metavar="K",
                    help="replace the block eigensolver and its spectrum by K Lanczos-Haydock "
                         "steps and the continued-fraction eps2 (no eigenvalues)")
    ap.add_argument("--nrefine", type=int, default=0, metavar="K",
                    help="FP64 refinement of the lowest K block eigenvalues (0..256)")
    ap.add_argument("--forms", type=int, default=-1, metavar="K",
                    help="after the timed steps, time K solves each of the refined split-BF16 "
                         "form and of the plain FP64 form, every solve checked against the "
                         "oracle's stored solution (default: 3 for cfg3, else 0)")
    ap.add_argument("--profile-all", action="store_true",
                    help="time every kernel (adds event records; breakdown on stderr)")
    args = ap.parse_args()
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the block eigensolver keeps each block on one device); use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.sync_probe:
        from paper_2603_24860_amd import bse as B
        props = torch.cuda.get_device_properties(0)
        out = {"device": props.name, "compute_units": props.multi_processor_count,
               "steps": args.sync_probe, "us_per_step": {}}
        buf = torch.zeros(2 * 4096, dtype=torch.int32, device="cuda")
        for wgs in (256, 512, 1024):
            row = {}
            for mode, name in ((0, "launch_per_step"), (1, "grid_barrier")):
                B.bse_sync_probe(mode, wgs, 100, buf)  # warm-up
                row[name] = round(B.bse_sync_probe(mode, wgs, args.sync_probe, buf), 3)
            out["us_per_step"][str(wgs)] = row
        print(json.dumps(out), flush=True)
        return
    if args.copy_mib:
        src = torch.ones(args.copy_mib * 2**18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out = {"copy_bytes": src.numel() * 4, "launches": 3}
        if args.copy_timed > 0:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.copy_timed):
                dst.copy_(src)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.copy_timed
            out.update(launches=3 + args.copy_timed, timed=args.copy_timed,
                       us_per_copy=round(ms * 1e3, 2),
                       read_plus_write_TB_s=round(2 * src.numel() * 4 / (ms * 1e-3) / 1e12, 3))
        print(json.dumps(out), flush=True)
        return
    import synth
    import workloads
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.system import Solver
    if args.workload == "cfg4":
        return bench_batched(args)
    if args.workload in ("cfg5", "cfg5l", "cfg5w"):
        return bench_served(args, large=args.workload == "cfg5l", wide=args.workload == "cfg5w")

    prec = {"fp32": B.FP32, "fp64": B.FP64, "bf16x3": B.BF16X3}[args.prec]
    cfg = synth.config(args.workload)
    ref = None if args.partner else oracle_reference(args.workload)
    t0 = time.perf_counter()
    host = workloads.host_inputs(cfg)
    log(f"inputs drawn in {time.perf_counter() - t0:.1f} s")
    S = make_system(cfg, host, prec)
    if args.seed_direct and not args.seed:
        print("--seed-direct needs --seed", file=sys.stderr)
        sys.exit(2)
    if args.seed:
        S.use_seed(direct=args.seed_direct)
    irrep, weights = S.active_irrep()
    if ref is not None and ref["irrep"] != irrep:
        ref = None
    sv = Solver(S, irrep, partner=0 if args.partner else None, nrefine=args.nrefine)
    n_block = sv.blk.n
    log(f"setup {time.perf_counter() - t0:.1f} s; N = {S.N}, block {irrep}"
        f"{' x-partner' if args.partner else ''} n = {sv.blk.n}")
    if ref is not None:  # the oracle's frequency grid
        sv.set_grid(np.linspace(ref["wmin"], ref["wmax"], ref["nw"]))
        sv.step()
    else:  # frequency grid from the block spectrum (first solve, untimed)
        sv.step()
        torch.cuda.synchronize()
        om = sv.omega.cpu().numpy()
        sv.set_grid(synth.omega_grid_from_range(om.min(), om.max()))
    for _ in range(args.warmup):
        sv.step()
    torch.cuda.synchronize()
    if args.haydock:  # the eigenpair eps2 on the same grid, to compare against
        eps2_eigh = sv.eps2.clone()
        for _ in range(max(1, args.warmup)):
            sv.haydock(args.haydock)
        torch.cuda.synchronize()

    B.bse_prof_enable("k_" if args.profile_all else "k_direct")
    B.bse_prof_reset()
    B.bse_prof_collect()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5 * args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        e = ev[5 * s:5 * s + 5]
        e[0].record()
        S.build()
        e[1].record()
        sv.project()
        e[2].record()
        if args.haydock:
            sv.haydock_steps(args.haydock)
            e[3].record()
            sv.haydock_spectrum()
        else:
            sv.eigh()
            e[3].record()
            sv.spectrum()
            if args.eels:
                sv.longitudinal()
        e[4].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = B.bse_prof_collect()
    B.bse_prof_enable(None)
    stages = np.array([[ev[5 * s + i].elapsed_time(ev[5 * s + i + 1]) for i in range(4)]
                       for s in range(args.steps)])
    st_ms = stages.mean(axis=0)
    nk, nv, nc, nmb = S.nk, S.nv, S.nc, S.nmb
    s1, s2, ex = build_flops(nk, nv, nc, nmb)
    if args.seed:  # contractions performed: one pair per pair orbit, one k per k orbit
        dims = B.bse_dims_get(S.group, S.grid)
        s1, s2 = s1 * dims["nporb"] / nk ** 2, s2 * dims["nporb"] / nk ** 2
        ex = ex * (dims["nkorb"] / nk) ** 2
    build_tflops = (s1 + s2 + ex) / (st_ms[0] * 1e-3) / 1e12
    ms_step = wall * 1e3 / args.steps
    fused = [k for k in ("k_direct_seed", "k_direct_fused", "k_direct_bf3") if k in prof]
    kname = fused[0] if fused else "k_direct_t"
    kt_ms, kt_n = prof.get(kname, (float("nan"), 0))
    kflops = (s1 + s2) if fused else s1   # flops of the kernel per build
    achieved = kflops * args.steps / (kt_ms * 1e-3) / 1e12 if kt_n else None
    res = sv.results()
    pk = PEAK[args.prec]
    out = {
        "metric": "H-build TFLOP/s + block-eigh s; solves/s & p99 latency at 0.1 meV vs FP64",
        "value": round(build_tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "fp32", "fp64": "fp64", "bf16x3": "bf16x3"}[args.prec],
        "data": "synthetic (seeded; paper-shaped Oh system, random-phase pair vectors)",
        "config": {"workload": f"{cfg['name']}: Oh {cfg['grid'][0]}x{cfg['grid'][1]}x"
                               f"{cfg['grid'][2]} k grid ({nk} k), Nv={nv}, Nc={nc}, N={S.N}, "
                               f"Nmb={nmb}, dipole-active {irrep}"
                               f"{' x-partner' if args.partner else ''} block n={sv.blk.n}, "
                               + ("eps2 and loss spectrum (secular equation), " if args.eels
                                  else "")
                               + (f"eps2 by {args.haydock} Lanczos-Haydock steps (no eigh), "
                                  if args.haydock else "")
                               + (f"seed build (one contraction per pair orbit)" if args.seed
                                  else f"dense-mode build of all {nk * nk} k pairs")
                               + (", block projected from the seed pieces (no H)"
                                  if args.seed_direct else ""),
                   "precision": args.prec, "nrefine": args.nrefine},
        "block_eigh_s": None if args.haydock else round(st_ms[2] * 1e-3, 6),
        "solves_per_s": round(1e3 / ms_step, 3),
        "stage_ms": {"build": round(st_ms[0], 3), "project": round(st_ms[1], 3),
                     ("haydock" if args.haydock else "block_eigh"): round(st_ms[2], 3),
                     ("spectrum+eels" if args.eels else "spectrum"): round(st_ms[3], 3)},
        "lowest_exciton_eV": [round(float(x), 9) for x in res["lowest"][:3]],
        "roofline": {
            "kernel": kname + (" (direct term, both contractions: W(q) Mv and conj(Mc) T, "
                               "complex MFMA" + (", split BF16: 3 bf16 products per product, "
                                                 "peak = bf16 dense / 3" if
                                                 kname == "k_direct_bf3" else "") + ")"
                               if fused else ""),
            "bound": "mfma",
            "achieved": round(achieved, 3) if achieved else None,
            "peak": pk,
            "unit": "TFLOP/s",
            "frac": round(achieved / pk, 4) if achieved else None,
            "traffic": measured_traffic(args.workload, args.prec, args.seed),
            "traffic_unit": "B/launch (HBM fetch + write, rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                            "copy-calibrated)",
            "flops_per_launch": kflops / max(1, kt_n // args.steps),
            "avg_launch_ms": kt_ms / kt_n if kt_n else None,
        },
    }
    if ref is not None and not args.haydock:
        err, e2err = accuracy(res, ref)
        bar = BARS["fp64" if args.prec == "fp64" else
                   ("bf16x3" if args.prec == "bf16x3" and args.nrefine > 0 else "fp32")]
        out["accuracy_vs_oracle"] = {"lowest100_max_err_eV": err, "eps2_rel_err": e2err,
                                     "bar_eV": bar, "meets_bars": bool(err < bar and
                                                                       e2err <= EPS2_BAR)}
        log(f"against the oracle: lowest-100 max err {err:.2e} eV, eps2 rel err {e2err:.2e}")
    if args.haydock:
        dev = float((sv.hd_eps2 - eps2_eigh).abs().max() / eps2_eigh.abs().max())
        out["haydock"] = {"K": args.haydock, "eps2_rel_dev_vs_eigh": dev}
    if args.eels:
        xo = sv.xosc.cpu().numpy()
        xp = sv.xpole.cpu().numpy()[xo > 0]
        out["lowest_longitudinal_eV"] = [round(float(x), 9) for x in xp[:3]]
    if args.profile_all:
        for k, (ms, n) in sorted(prof.items(), key=lambda x: -x[1][0]):
            log(f"  {k:14s} {ms / args.steps:10.3f} ms/step  {n // args.steps:6d} launches/step")
    nforms = args.forms if args.forms >= 0 else (3 if args.workload == "cfg3" else 0)
    if nforms and ref is not None and not (args.partner or args.seed or args.haydock):
        sv.s.H = None  # free the timed form's H and build workspace first
        sv.s.ws = None
        del sv, S
        torch.cuda.empty_cache()
        out["precision_forms"] = precision_forms(cfg, host, irrep, nforms, ref, log)
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, n_block, log)
    print(json.dumps(out), flush=True)


def make_system(cfg, host, prec):
    from paper_2603_24860_amd.system import DeviceSystem
    group, grid, T, inputs = host
    return DeviceSystem(group, grid, cfg["nv"], cfg["nc"], cfg["nmb"], T, inputs, prec)


def precision_forms(cfg, host, irrep, nsolve, ref, log_fn):
    """The refined split-BF16 form (split-BF16 build, FP32 eigensolver, FP64
    refinement of the lowest 100) against the plain FP64 GPU form (FP64 build,
    projection, eigensolver and spectrum): each timed over nsolve whole solves
    (inputs resident in HBM, lowest 100 energies and eps2 copied to the host),
    every solve checked against the oracle's stored solution.  solves/s at
    0.1 meV counts only the solves within 0.1 meV (lowest 100) and 1e-4 (eps2)."""
    import torch
    from paper_2603_24860_amd import bse as B
    from paper_2603_24860_amd.system import Solver
    wgrid = np.linspace(ref["wmin"], ref["wmax"], ref["nw"])
    out = {}
    for name, prec, nref in (("refined_bf16x3", B.BF16X3, 100), ("plain_fp64", B.FP64, 0)):
        S = make_system(cfg, host, prec)
        sv = Solver(S, irrep, nrefine=nref, wgrid=wgrid)
        sv.step()
        sv.results()
        errs, e2s, ok = [], [], 0
        t0 = time.perf_counter()
        for _ in range(nsolve):
            sv.step()
            res = sv.results()
            err, e2 = accuracy(res, ref)
            errs.append(err)
            e2s.append(e2)
            ok += int(err <= 1e-4 and e2 <= EPS2_BAR)
        wall = time.perf_counter() - t0
        out[name] = {"solves": nsolve, "ms_per_solve": round(wall * 1e3 / nsolve, 3),
                     "solves_per_s": round(nsolve / wall, 4),
                     "solves_within_0.1meV": ok,
                     "solves_per_s_at_0.1meV": round(ok / wall, 4),
                     "max_lowest100_err_meV": max(errs) * 1e3, "max_eps2_rel_err": max(e2s),
                     "nrefine": nref}
        log_fn(f"{name}: {wall * 1e3 / nsolve:.1f} ms per solve, lowest-100 max err "
               f"{max(errs) * 1e3:.2e} meV, eps2 {max(e2s):.2e}, {ok}/{nsolve} within the bars")
        S.H = None
        S.ws = None
        del sv, S
        torch.cuda.empty_cache()
    f = out["plain_fp64"]["solves_per_s_at_0.1meV"]
    out["refined_bf16x3_over_plain_fp64_at_0.1meV"] = (
        round(out["refined_bf16x3"]["solves_per_s_at_0.1meV"] / f, 3) if f > 0 else None)
    return out


if __name__ == "__main__":
    main()
