"""k grid, group action on it, and the orbits used by the symmetry treatment.

Paper: Eq. (sk) (s k = A k folded back into the Brillouin zone); Sec. III.C.2
(the loop over q is outermost; pairs (k, k') related by one operation share
their matrix elements); Sec. III.C.4 (the projector acts within the orbit of a
product function).

Conventions: k lin = (k1 n2 + k2) n3 + k3; pair lin = k nk + k'; q = k - k'
(mod grid).  Orbit ids are assigned in increasing order of the orbit's
canonical representative, the smallest linear index in it.
"""
import numpy as np


def kgrid(grid):
    n1, n2, n3 = grid
    k = np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)],
                 dtype=np.int64)
    return k


def lin(grid, k):
    n1, n2, n3 = grid
    return (k[..., 0] * n2 + k[..., 1]) * n3 + k[..., 2]


def kperm(grid, kmat):
    """kperm[s, k] = lin((A_s k) mod grid) for every op s and grid point k."""
    k = kgrid(grid)
    g = np.asarray(grid)
    out = np.empty((len(kmat), len(k)), dtype=np.int64)
    for s, A in enumerate(kmat):
        out[s] = lin(grid, np.mod(k @ A.T, g))
    # the group must map the grid onto itself (e.g. Oh needs n1 = n2 = n3)
    if not all(len(np.unique(row)) == len(k) for row in out):
        raise ValueError(f"the point group does not act on the {tuple(grid)} grid")
    return out


def qindex(grid):
    """qidx[k, k'] = lin(k - k' mod grid)."""
    k = kgrid(grid)
    g = np.asarray(grid)
    d = np.mod(k[:, None, :] - k[None, :, :], g)
    return lin(grid, d)


def orbits_of(perm_min_key, keys):
    """Canonical representative (minimum key over the group) and dense ids."""
    reps = perm_min_key
    uniq = np.unique(reps)
    ids = np.searchsorted(uniq, reps)
    return uniq, ids


def k_orbits(kp):
    """k orbits: rep[k] (min lin index over s k), orbit id, list of reps."""
    rep = kp.min(axis=0)
    uniq, ids = orbits_of(rep, None)
    return uniq, ids, rep


def pair_orbits(kp):
    """Orbits of (k, k') under the diagonal action (s k, s k').

    Returns (reps[nporb], porb[nk*nk]) with reps the minimum pair lin index.
    """
    nops, nk = kp.shape
    best = None
    for s in range(nops):
        key = kp[s][:, None] * nk + kp[s][None, :]
        best = key if best is None else np.minimum(best, key)
    best = best.reshape(-1)
    uniq, ids = orbits_of(best, None)
    return uniq, ids


def pair_classes(nk, preps, porb):
    """Swap partners and storage classes of pair orbits.

    swap(p) = orbit of (k', k) for (k, k') in p.  Class = {p, swap(p)}, stored
    once in the orientation of the smaller orbit id; classes are numbered in
    increasing order of that id.
    Returns swap[nporb], cls_of_orbit[nporb], conj_of_orbit[nporb] (orbit is the
    larger member, so its data is the band conjugate transpose of the stored one),
    class_rep_pair[ncls], class_selfswap[ncls].
    """
    k = preps // nk
    kq = preps % nk
    swap = porb[kq * nk + k]
    lo = np.minimum(np.arange(len(preps)), swap)
    owners = np.unique(lo)
    cls_of = np.searchsorted(owners, lo)
    conj_of = (np.arange(len(preps)) > swap).astype(np.uint8)
    return swap, cls_of, conj_of, preps[owners], swap[owners] == owners


def tables(grid, kmat):
    """All integer tables for one system (dict of numpy arrays)."""
    kp = kperm(grid, kmat)
    nk = kp.shape[1]
    kreps, korb, krep_of_k = k_orbits(kp)
    preps, porb = pair_orbits(kp)
    swap, cls_of, conj_of, class_rep, class_ss = pair_classes(nk, preps, porb)
    qidx = qindex(grid).reshape(-1)
    return dict(
        grid=tuple(grid), nk=nk, kperm=kp,
        nkorb=len(kreps), korb_reps=kreps, korb=korb, krep_of_k=krep_of_k,
        nporb=len(preps), porb_reps=preps, porb=porb, pswap_partner=swap,
        ncls=len(class_rep), class_rep=class_rep, class_selfswap=class_ss,
        pidx=cls_of[porb], pconj=conj_of[porb],
        qidx=qidx, qorb=korb,  # q orbits are the k orbits of the same grid
    )
