"""Counter-based generator and the synthetic workload recipe.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a hash of a key built
from (seed, tensor tag, indices).  A draw therefore depends only on the key,
never on the order in which arrays are enumerated.

Recipe (all energies in eV):
  * E_v(k) = -0.6 - 0.1 f(k) + jitter,  E_c(k) = 0.6 + 0.2 (3 - f(k)) + jitter,
    f = sum_i cos(2 pi k_i / n) on cubic grids and the hexagonal star sum
    cos 2pi k1 + cos 2pi k2 + cos 2pi (k1 + k2) on hexagonal grids, so that E is
    invariant under the point group; jitter ~ N(0, 0.01^2) per (k orbit, band).
  * v_I = 4 pi / (I + 1)  (diagonal bare Coulomb matrix in the mixed basis).
  * Pair vectors: complex Gaussian with E|z|^2 = exp(-I/16), drawn per orbit
    (k orbit for the exchange vectors, pair-orbit class for the direct ones).
    A class whose orbit is its own swap partner is made band-Hermitian.
  * W(q) = v^1/2 (1 + chi)^-1 v^1/2 with chi = G G^T, G real N x 8 with entries
    N(0, 1/N), drawn per q orbit.
  * Dipoles: per k orbit a complex Gaussian 3-vector g (or scalar), expanded
    to every k of the orbit equivariantly: d(k) = mean over the ops s with
    s r = k of R_s g, r the orbit representative.  B = e . d.
"""
import math
import os
import numpy as np

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_GOLD = np.uint64(0x9E3779B97F4A7C15)

# tensor tags: fixed small integers so keys never collide across tensors
TAG = {"ejv": 1, "ejc": 2, "mx": 3, "mv": 4, "mc": 5, "chi": 6, "dip": 7, "batch": 8}


def splitmix64(z):
    """SplitMix64 output function applied elementwise to uint64 state z+gamma."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLD
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _key(seed, tag, *idx):
    """Chain-hash (seed, tag, i0, i1, ...) with broadcasting over index arrays."""
    h = splitmix64(np.uint64(seed) * np.uint64(1) + np.uint64(TAG[tag]) * np.uint64(1 << 40))
    for i in idx:
        with np.errstate(over="ignore"):
            h = splitmix64(h ^ (np.asarray(i, dtype=np.int64).astype(np.uint64) * _GOLD))
    return h


def keyed_uniform(seed, tag, *idx, draw=0):
    """Uniform on [0,1) with 53 random bits; `draw` selects an independent stream."""
    with np.errstate(over="ignore"):
        h = splitmix64(_key(seed, tag, *idx) + np.uint64(draw) * np.uint64(0xD1B54A32D192ED03))
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def keyed_complex(seed, tag, *idx, var=1.0):
    """Complex Gaussian with E|z|^2 = var (Box-Muller on two keyed uniforms)."""
    u1 = 1.0 - keyed_uniform(seed, tag, *idx, draw=0)
    u2 = keyed_uniform(seed, tag, *idx, draw=1)
    r = np.sqrt(-2.0 * np.log(u1)) * np.sqrt(np.asarray(var) / 2.0)
    return r * np.cos(2 * np.pi * u2) + 1j * (r * np.sin(2 * np.pi * u2))


def keyed_normal(seed, tag, *idx, std=1.0):
    """Real Gaussian N(0, std^2) (real part of a unit Box-Muller pair, rescaled)."""
    u1 = 1.0 - keyed_uniform(seed, tag, *idx, draw=0)
    u2 = keyed_uniform(seed, tag, *idx, draw=1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2 * np.pi * u2) * std


# ----------------------------------------------------------------------------
# workload configurations (sizes of the paper-shaped synthetic systems)
# ----------------------------------------------------------------------------
CONFIGS = {
    # name: lattice, grid, nv, nc, nmb, seed, build precision
    "cfg1": dict(lattice="cubic", grid=(4, 4, 4), nv=3, nc=3, nmb=64, seed=1),
    "cfg2": dict(lattice="cubic", grid=(8, 8, 8), nv=4, nc=4, nmb=256, seed=2),
    "cfg3": dict(lattice="cubic", grid=(12, 12, 12), nv=4, nc=6, nmb=384, seed=3),
}
ETA = 0.05       # Lorentzian broadening in eV
NOMEGA = 2000    # points on the frequency grid


def batch_configs(seed=4, count=64):
    """The batched workload: `count` layered hexagonal (D6h) systems.  Seed 4
    draws each system's shape (n x n x 1 grid with n in 6..24, Nv and Nc in
    2..4, Nmb in {128, 192, 256, 320}); system s draws its data with seed
    4000 + s, so systems of equal shape still differ."""
    out = []
    for s in range(count):
        u = [float(keyed_uniform(seed, "batch", s, j)) for j in range(4)]
        n = 6 + int(u[0] * 19)
        out.append(dict(lattice="hex", grid=(n, n, 1), nv=2 + int(u[1] * 3), nc=2 + int(u[2] * 3),
                        nmb=(2 + int(u[3] * 4)) * 64, seed=4000 + s, name=f"cfg4.{s}"))
    return out


def config(name, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    c["name"] = name
    return c


def band_energies(seed, lattice, grid, kfrac, rep_of_k, nv, nc, jitter=0.01):
    """E_v[nk, nv], E_c[nk, nc] in eV.

    kfrac[nk, 3]: k in reduced coordinates (k_i / n_i); rep_of_k[nk]: the linear
    index of the orbit representative of each k (keys the per-orbit jitter).
    """
    kfrac = np.asarray(kfrac, dtype=np.float64)
    c = np.cos(2 * np.pi * kfrac)
    if lattice == "cubic":
        f = c.sum(axis=1)
    elif lattice == "hex":
        f = c[:, 0] + c[:, 1] + np.cos(2 * np.pi * (kfrac[:, 0] + kfrac[:, 1]))
    else:
        raise ValueError(lattice)
    rep = np.asarray(rep_of_k, dtype=np.int64)
    bv = np.arange(nv)
    bc = np.arange(nc)
    jv = keyed_normal(seed, "ejv", rep[:, None], bv[None, :], std=jitter)
    jc = keyed_normal(seed, "ejc", rep[:, None], bc[None, :], std=jitter)
    ev = -0.6 - 0.1 * f[:, None] + jv
    ec = 0.6 + 0.2 * (3.0 - f[:, None]) + jc
    return ev, ec


def coulomb_diag(nmb):
    return 4 * np.pi / (np.arange(nmb, dtype=np.float64) + 1.0)


def exchange_vectors(seed, korb_reps, nv, nc, nmb):
    """M_x per k orbit: [nkorb, nv, nc, nmb] complex128."""
    r = np.asarray(korb_reps, dtype=np.int64)[:, None, None, None]
    v = np.arange(nv)[None, :, None, None]
    c = np.arange(nc)[None, None, :, None]
    i = np.arange(nmb)[None, None, None, :]
    return keyed_complex(seed, "mx", r, v, c, i, var=np.exp(-i / 16.0))


def pair_vectors(seed, tag, class_reps, class_selfswap, nb, nmb, chunk=1024, threads=16):
    """M_v or M_c per pair class: [ncls, nb, nb, nmb] complex128.

    class_reps[ncls]: linear pair index k*nk+k' of the stored orientation;
    class_selfswap[ncls]: the class's orbit is its own swap partner, so the
    stored matrix must equal its conjugate transpose over the band indices.
    Chunks of classes are drawn in parallel threads (numpy releases the GIL in
    its array kernels); every value depends only on its key, so the result does
    not depend on the chunking or the thread count.
    """
    reps = np.asarray(class_reps, dtype=np.int64)
    ss = np.asarray(class_selfswap, dtype=bool)
    out = np.empty((len(reps), nb, nb, nmb), dtype=np.complex128)
    b1 = np.arange(nb)[None, :, None, None]
    b2 = np.arange(nb)[None, None, :, None]
    i = np.arange(nmb)[None, None, None, :]
    var = np.exp(-i / 16.0)

    def fill(s):
        r = reps[s:s + chunk][:, None, None, None]
        z = keyed_complex(seed, tag, r, b1, b2, i, var=var)
        sel = ss[s:s + chunk]
        if sel.any():
            zs = z[sel]
            z[sel] = (zs + np.conj(np.swapaxes(zs, 1, 2))) / math.sqrt(2.0)
        out[s:s + chunk] = z

    starts = range(0, len(reps), chunk)
    nt = max(1, min(threads, len(starts), os.cpu_count() or 1))
    if nt == 1:
        for s in starts:
            fill(s)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(fill, starts))
    return out


def screened_w(seed, qorb_reps, nmb, rank=8):
    """W per q orbit: [nqorb, nmb, nmb] real symmetric."""
    v = coulomb_diag(nmb)
    sv = np.sqrt(v)
    out = np.empty((len(qorb_reps), nmb, nmb))
    I = np.arange(nmb)[:, None]
    R = np.arange(rank)[None, :]
    for n, q in enumerate(qorb_reps):
        G = keyed_normal(seed, "chi", q, I, R, std=1.0 / math.sqrt(nmb))
        chi = G @ G.T
        inv = np.linalg.inv(np.eye(nmb) + chi)
        inv = 0.5 * (inv + inv.T)
        out[n] = sv[:, None] * inv * sv[None, :]
    return out


def dipoles(seed, kperm, rcart, rep_of_k, nv, nc, pol=(1.0, 0.0, 0.0), vector=True):
    """Dipole projections B[nk, nv, nc] complex.

    kperm[nops, nk]: index of s k; rcart[nops, 3, 3]: Cartesian matrix of each op;
    rep_of_k[nk]: linear index of each k's orbit representative.
    vector=True draws a 3-vector per (orbit, v, c) and expands it equivariantly
    (d(s r) = R_s d(r), d(r) averaged over the stabiliser of r); vector=False
    draws a scalar per (orbit, v, c), copied to the whole orbit.
    """
    kperm = np.asarray(kperm)
    rep = np.asarray(rep_of_k, dtype=np.int64)
    nk = kperm.shape[1]
    v = np.arange(nv)[None, :, None]
    c = np.arange(nc)[None, None, :]
    if not vector:
        return keyed_complex(seed, "dip", rep[:, None, None], v, c, 0)
    pol = np.asarray(pol, dtype=np.float64)
    d = np.zeros((nk, nv, nc, 3), dtype=np.complex128)
    cnt = np.zeros(nk)
    reps = np.unique(rep)
    g = np.stack([keyed_complex(seed, "dip", reps[:, None, None], v, c, 1 + x)
                  for x in range(3)], axis=-1)            # [nrep, nv, nc, 3]
    gi = {int(r): j for j, r in enumerate(reps)}
    for s in range(kperm.shape[0]):
        for r in reps:
            k = kperm[s, r]
            d[k] += np.einsum("ij,vcj->vci", rcart[s], g[gi[int(r)]])
            cnt[k] += 1
    d /= cnt[:, None, None, None]
    return np.einsum("kvcx,x->kvc", d, pol)


def omega_grid_from_range(wmin, wmax, eta=ETA, npts=NOMEGA):
    """Uniform frequency grid covering [wmin - 10 eta, wmax + 10 eta]."""
    return np.linspace(wmin - 10 * eta, wmax + 10 * eta, npts)
