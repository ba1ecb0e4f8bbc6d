"""FP64 oracle of the Tamm-Dancoff BSE hot path: H, projection, eigh, spectrum.

Paper passages followed (REVTeX source, equations by label):
  * Eq. (BSE-eigval): H = (e_ku - e_ko) delta + vbar-term - W-term, Hermitian in
    the Tamm-Dancoff approximation (Sec. II, last paragraph); spin factor 2 in
    front of vbar for a non-magnetic system without spin-orbit coupling.
  * Eq. (w_interaction2): each interaction element is a vector-matrix-vector
    product over the mixed-basis index with prefactor 1/N_k.
  * Eq. (projection), Sec. III.C.4: P_mu = d_mu/|S| sum_s chi_mu(s)* Gamma(s),
    applied to unit vectors orbit by orbit and orthonormalised by SVD; U_mu
    collects the vectors, H_mu = U_mu^dag H U_mu (Eq. (transformationU)).
  * Eqs. (macro_diel), (reducible_polar), (oscillatorA): eps2(w) =
    (8 pi / N_k) sum_l |B_l|^2 [L(w - W_l) + L(w + W_l)], L(x) = eta/(x^2+eta^2),
    with the spin factor 2 and V_uc = 1.

Index layout: a = (k nv + v) nc + c.  Block layout of H_mu: orbits in id order,
then the orbit's basis vectors, then (v, c) with c fastest.
"""
import numpy as np

import synth
from . import groups, orbits


# ----------------------------------------------------------------------------
# problem assembly: the oracle's own tables feed the shared input generator
# ----------------------------------------------------------------------------
class _ClassSubset:
    """M_v or M_c for a subset of swap classes, indexed by class id.

    The generator keys every draw by the class's representative pair, so the
    subset holds exactly the values the full array would hold for those ids."""

    def __init__(self, ids, M):
        self.pos = {int(c): i for i, c in enumerate(ids)}
        self.M = M

    def __getitem__(self, cls):
        cls = np.atleast_1d(np.asarray(cls))
        return self.M[np.array([self.pos[int(c)] for c in cls.ravel()])].reshape(
            cls.shape + self.M.shape[1:])


def make_problem(cfg, vector_dipole=True, zero_interaction=False, pairs=None):
    """Tables (oracle's own) plus seeded inputs for one synthetic system.

    pairs: optional iterable of k-pair ids k N_k + k'; M_v and M_c are then
    drawn only for the swap classes of those pairs, which is enough for the
    single elements H[(k,v,c), (k',v',c')] of a large system."""
    lattice = cfg.get("lattice", "cubic")
    g = groups.group("Oh" if lattice == "cubic" else "D6h")
    grid = tuple(cfg["grid"])
    T = orbits.tables(grid, g["kmat"])
    nv, nc, nmb, seed = cfg["nv"], cfg["nc"], cfg["nmb"], cfg["seed"]
    kfrac = orbits.kgrid(grid) / np.asarray(grid, dtype=np.float64)
    ev, ec = synth.band_energies(seed, lattice, grid, kfrac, T["krep_of_k"], nv, nc)
    vd = synth.coulomb_diag(nmb)
    mx = synth.exchange_vectors(seed, T["korb_reps"], nv, nc, nmb)
    if pairs is None:
        mv = synth.pair_vectors(seed, "mv", T["class_rep"], T["class_selfswap"], nv, nmb)
        mc = synth.pair_vectors(seed, "mc", T["class_rep"], T["class_selfswap"], nc, nmb)
    else:
        ids = np.unique(T["pidx"][np.asarray(list(pairs), dtype=np.int64)])
        reps, ss = T["class_rep"][ids], T["class_selfswap"][ids]
        mv = _ClassSubset(ids, synth.pair_vectors(seed, "mv", reps, ss, nv, nmb))
        mc = _ClassSubset(ids, synth.pair_vectors(seed, "mc", reps, ss, nc, nmb))
    w = synth.screened_w(seed, T["korb_reps"], nmb)
    B = synth.dipoles(seed, T["kperm"], g["rcart"], T["krep_of_k"], nv, nc,
                      vector=vector_dipole).reshape(-1)
    if zero_interaction:
        vd = np.zeros_like(vd)
        w = np.zeros_like(w)
    return dict(cfg=cfg, group=g, T=T, nk=T["nk"], nv=nv, nc=nc, nmb=nmb,
                N=T["nk"] * nv * nc, ev=ev, ec=ec, vdiag=vd, mx=mx, mv=mv, mc=mc,
                w=w, B=B)


def pair_block(P, name, k, kq):
    """M_name(k, k') for arrays k, k' (gathered from the class storage)."""
    T = P["T"]
    nk = P["nk"]
    p = k * nk + kq
    M = P[name][T["pidx"][p]]
    cj = T["pconj"][p].astype(bool)
    if cj.any():
        M = M.copy()
        M[cj] = np.conj(np.swapaxes(M[cj], 1, 2))
    return M


# ----------------------------------------------------------------------------
# H, Eq. (BSE-eigval) with Eq. (w_interaction2)
# ----------------------------------------------------------------------------
def diagonal(P):
    """(e_c(k) - e_v(k)) on the diagonal, a = (k nv + v) nc + c."""
    return (P["ec"][:, None, :] - P["ev"][:, :, None]).reshape(-1)


def exchange(P):
    """2/N_k sum_I M_x[k,v,c,I] v_I conj(M_x[k',v',c',I])  (N x N)."""
    T = P["T"]
    Mx = P["mx"][T["korb"]].reshape(P["N"], P["nmb"])
    return (2.0 / P["nk"]) * (Mx * P["vdiag"][None, :]) @ Mx.conj().T


def direct(P, qs=None):
    """1/N_k sum_IJ conj(M_c[k,k'][c,c',I]) W_IJ(k-k') M_v[k,k'][v,v',J]  (N x N).

    Loop over q outermost (Sec. III.C.2), all k for each q.  `qs` restricts the
    loop to a subset of q (the other pairs stay zero); used to time a sample.
    """
    nk, nv, nc = P["nk"], P["nv"], P["nc"]
    T = P["T"]
    D = np.zeros((nk, nv, nc, nk, nv, nc), dtype=np.complex128)
    qidx = T["qidx"].reshape(nk, nk)
    kk = np.arange(nk)
    for q in (range(nk) if qs is None else qs):
        kq = np.array([int(np.nonzero(qidx[k] == q)[0][0]) for k in kk])  # k' = k - q
        W = P["w"][T["qorb"][q]]
        Mv = pair_block(P, "mv", kk, kq)       # [nk, nv, nv, nmb]
        Mc = pair_block(P, "mc", kk, kq)       # [nk, nc, nc, nmb]
        Tq = Mv @ W.T                           # sum_J W_IJ Mv[..., J]
        Dq = np.einsum("kcdi,kvwi->kvcwd", Mc.conj(), Tq)
        D[kk, :, :, kq, :, :] = Dq
    return D.reshape(P["N"], P["N"]) / nk


def hamiltonian(P):
    """Full unsymmetrised H (complex128, N x N)."""
    H = exchange(P) - direct(P)
    H[np.diag_indices_from(H)] += diagonal(P)
    return H


def hamiltonian_element(P, a, b):
    """H[a, b] straight from the definition, one element at a time."""
    nv, nc, nk = P["nv"], P["nc"], P["nk"]
    T = P["T"]
    k, v, c = a // (nv * nc), (a // nc) % nv, a % nc
    k2, v2, c2 = b // (nv * nc), (b // nc) % nv, b % nc
    val = 0j
    if a == b:
        val += P["ec"][k, c] - P["ev"][k, v]
    mx1 = P["mx"][T["korb"][k], v, c]
    mx2 = P["mx"][T["korb"][k2], v2, c2]
    val += (2.0 / nk) * np.sum(mx1 * P["vdiag"] * np.conj(mx2))
    Mv = pair_block(P, "mv", np.array([k]), np.array([k2]))[0]
    Mc = pair_block(P, "mc", np.array([k]), np.array([k2]))[0]
    W = P["w"][T["qorb"][T["qidx"][k * nk + k2]]]
    val -= (1.0 / nk) * (np.conj(Mc[c, c2]) @ W @ Mv[v, v2])
    return val


# ----------------------------------------------------------------------------
# symmetry-adapted basis, Eq. (projection) and Eq. (transformationU)
# ----------------------------------------------------------------------------
def orbit_members(P):
    T = P["T"]
    return [np.nonzero(T["korb"] == o)[0] for o in range(T["nkorb"])]


def orbit_projector(P, chi, d, members):
    """P_mu restricted to the k orbit (the band indices are spectators)."""
    kp = P["T"]["kperm"]
    pos = {int(k): i for i, k in enumerate(members)}
    m = len(members)
    Pm = np.zeros((m, m))
    for s in range(kp.shape[0]):
        for i, k in enumerate(members):
            Pm[pos[int(kp[s, k])], i] += chi[s]
    return Pm * (d / kp.shape[0])


def isotypic_basis(P, irrep_name):
    """Per-orbit orthonormal bases of the irrep's isotypic subspace.

    Returns dict(n, orb_off[nkorb], orb_dim[nkorb], basis=list of (members, U_O)).
    orb_dim[O] = d_mu m_mu(O), the rank of P_mu on the orbit.
    """
    d, chi = groups.irrep(P["group"], irrep_name)
    nb = P["nv"] * P["nc"]
    mem = orbit_members(P)
    offs, dims, basis = [], [], []
    off = 0
    for o, members in enumerate(mem):
        Pm = orbit_projector(P, chi, d, members)
        u, s, _ = np.linalg.svd(Pm)
        r = int(np.sum(s > 0.5))
        offs.append(off)
        dims.append(r)
        basis.append((members, u[:, :r]))
        off += r * nb
    return dict(irrep=irrep_name, d=d, n=off, orb_off=np.array(offs, dtype=np.int64),
                orb_dim=np.array(dims, dtype=np.int64), basis=basis)


# ----------------------------------------------------------------------------
# partner-resolved blocks of a vector irrep (a step beyond the paper, which uses
# characters only): for T1u of Oh and E1u, A2u of D6h the irrep matrices are
# the Cartesian rotation matrices R_s, so the projector onto row p is
#   P_pp = d/|S| sum_s (R_s)_{ii} Gamma(s),  i = the Cartesian axis of row p
# ----------------------------------------------------------------------------
VECTOR_ROWS = {"T1u": (0, 1, 2), "E1u": (0, 1), "A2u": (2,)}


def partner_weights(P, irrep_name, p):
    axis = VECTOR_ROWS[irrep_name][p]
    return P["group"]["rcart"][:, axis, axis]


def partner_basis(P, irrep_name, p):
    """Per-orbit orthonormal bases of the range of P_pp (same layout as
    isotypic_basis, orb_dim[O] = m_mu(O))."""
    d, _ = groups.irrep(P["group"], irrep_name)
    w = partner_weights(P, irrep_name, p)
    nb = P["nv"] * P["nc"]
    offs, dims, basis = [], [], []
    off = 0
    for members in orbit_members(P):
        Pm = orbit_projector(P, w, d, members)
        u, s, _ = np.linalg.svd(Pm)
        r = int(np.sum(s > 0.5))
        offs.append(off)
        dims.append(r)
        basis.append((members, u[:, :r]))
        off += r * nb
    return dict(irrep=irrep_name, d=d, n=off, orb_off=np.array(offs, dtype=np.int64),
                orb_dim=np.array(dims, dtype=np.int64), basis=basis)


def full_partner_projector(P, irrep_name, p):
    """Dense P_pp on the whole product space (small systems only)."""
    d, _ = groups.irrep(P["group"], irrep_name)
    w = partner_weights(P, irrep_name, p)
    kp = P["T"]["kperm"]
    nb = P["nv"] * P["nc"]
    Pm = np.zeros((P["N"], P["N"]))
    for s in range(kp.shape[0]):
        for k in range(P["nk"]):
            Pm[kp[s, k] * nb + np.arange(nb), k * nb + np.arange(nb)] += w[s]
    return Pm * (d / kp.shape[0])


def basis_matrix(P, blk):
    """Dense U_mu (N x n_mu) with the canonical block layout."""
    nv, nc = P["nv"], P["nc"]
    nb = nv * nc
    U = np.zeros((P["N"], blk["n"]))
    for o, (members, Uo) in enumerate(blk["basis"]):
        for j in range(Uo.shape[1]):
            for i, k in enumerate(members):
                U[k * nb:(k + 1) * nb, blk["orb_off"][o] + j * nb + np.arange(nb)] = \
                    np.eye(nb) * Uo[i, j]
    return U


def full_projector(P, irrep_name):
    """Dense P_mu on the whole product space (small systems only)."""
    d, chi = groups.irrep(P["group"], irrep_name)
    kp = P["T"]["kperm"]
    nb = P["nv"] * P["nc"]
    N = P["N"]
    Pm = np.zeros((N, N))
    for s in range(kp.shape[0]):
        for k in range(P["nk"]):
            Pm[kp[s, k] * nb + np.arange(nb), k * nb + np.arange(nb)] += chi[s]
    return Pm * (d / kp.shape[0])


def gamma_perm(P, s):
    """Gamma(s) as an index map: e_(k,v,c) -> e_(s k, v, c)."""
    nb = P["nv"] * P["nc"]
    kp = P["T"]["kperm"][s]
    return (kp[:, None] * nb + np.arange(nb)[None, :]).reshape(-1)


def block_dims_closed_form(P):
    """dim_mu = nv nc d_mu (1/|G|) sum_s chi_mu(s) fix(s) for every irrep."""
    kp = P["T"]["kperm"]
    fix = (kp == np.arange(P["nk"])[None, :]).sum(axis=1)
    out = {}
    for nm, d, chi in P["group"]["irreps"]:
        val = d * float(chi @ fix) / kp.shape[0]
        out[nm] = int(round(val)) * P["nv"] * P["nc"]
    return out


def project(H, U):
    return U.T @ H @ U


# ----------------------------------------------------------------------------
# the same H_mu without holding H: rows of H one k orbit at a time, each slab
# contracted with the per-orbit bases.  U_mu is block diagonal over k orbits
# (its columns for orbit O are U_O (x) I_bands on the rows of O, Eq.
# (transformationU)), so the rows of O meet only the block columns of O:
#   H_mu[O, O'] = (U_O (x) I)^T H[rows of O, rows of O'] (U_O' (x) I).
# For systems whose full H does not fit in host memory (N = 41472: 27.5 GB).
# ----------------------------------------------------------------------------
def _times_real(M, R):
    """M @ R for complex M (..., K) and real R (K x L): one real product over
    the real and imaginary parts of M, stacked as rows."""
    parts = np.ascontiguousarray(np.stack([M.real, M.imag], axis=-2))
    Y = (parts.reshape(-1, M.shape[-1]) @ R).reshape(M.shape[:-1] + (2, R.shape[1]))
    return Y[..., 0, :] + 1j * Y[..., 1, :]


def hamiltonian_rows(P, k, mx_all=None):
    """Rows a = (k, v, c) of H for one k against every column b (nb x N): the
    terms of hamiltonian() -- diagonal, exchange, direct -- for this slab."""
    nk, nv, nc, nmb, N = P["nk"], P["nv"], P["nc"], P["nmb"], P["N"]
    nb = nv * nc
    T = P["T"]
    if mx_all is None:
        mx_all = P["mx"][T["korb"]].reshape(N, nmb)
    # exchange: 2/N_k sum_I Mx[k,v,c,I] v_I conj(Mx[k',v',c',I])
    Hs = (2.0 / nk) * (mx_all[k * nb:(k + 1) * nb] * P["vdiag"][None, :]) @ mx_all.conj().T
    # direct: 1/N_k sum_IJ conj(Mc[k,k'][c,c',I]) W_IJ(k-k') Mv[k,k'][v,v',J]
    kk = np.full(nk, k)
    kq = np.arange(nk)
    Mv = pair_block(P, "mv", kk, kq)                   # [nk', nv, nv, nmb]
    Mc = pair_block(P, "mc", kk, kq)                   # [nk', nc, nc, nmb]
    qo = T["qorb"][T["qidx"][k * nk + kq]]             # q orbit of k - k'
    Tq = np.empty_like(Mv)
    for o in np.unique(qo):                            # one W(q) per q orbit
        sel = np.nonzero(qo == o)[0]
        Tq[sel] = _times_real(Mv[sel], P["w"][o].T)   # sum_J W_IJ Mv[..., J]
    D = np.matmul(Mc.conj().reshape(nk, nc * nc, nmb),
                  np.swapaxes(Tq.reshape(nk, nv * nv, nmb), 1, 2))  # [k', (c,c'), (v,v')]
    D = D.reshape(nk, nc, nc, nv, nv).transpose(3, 1, 0, 4, 2)    # [v, c, k', v', c']
    Hs -= D.reshape(nb, N) / nk
    Hs[np.arange(nb), k * nb + np.arange(nb)] += (P["ec"][k][None, :]
                                                  - P["ev"][k][:, None]).reshape(-1)
    return Hs


def orbit_slab(P, members, mx_all=None):
    """Rows of H for every k of one orbit: [|O|, nb, N]."""
    return np.stack([hamiltonian_rows(P, int(k), mx_all) for k in members])


def project_slab(P, blk, o, slab):
    """Row block of orbit o of H_mu from the orbit's H rows (orbit_slab):
    (U_O (x) I)^T H[rows of O, rows of O'] (U_O' (x) I) for every orbit O'."""
    nb = P["nv"] * P["nc"]
    members, Uo = blk["basis"][o]
    r = Uo.shape[1]
    out = np.zeros((r * nb, blk["n"]), dtype=np.complex128)
    slab = slab.reshape(len(members), nb, P["nk"], nb)
    for o2, (members2, Uo2) in enumerate(blk["basis"]):
        r2 = Uo2.shape[1]
        if r2 == 0:
            continue
        Hb = slab[:, :, members2, :]                               # [|O|, nb, |O'|, nb]
        Hb = np.einsum("ij,iakb,kl->jalb", Uo, Hb, Uo2, optimize=True)
        j0 = blk["orb_off"][o2]
        out[:, j0:j0 + r2 * nb] = Hb.reshape(r * nb, r2 * nb)
    return out


def project_streamed(P, blk, log=None):
    """H_mu = U_mu^T H U_mu (Eq. (transformationU)) for the block of
    isotypic_basis / partner_basis, forming H one k orbit of rows at a time."""
    nb = P["nv"] * P["nc"]
    mx_all = P["mx"][P["T"]["korb"]].reshape(P["N"], P["nmb"])
    Hm = np.zeros((blk["n"], blk["n"]), dtype=np.complex128)
    for o, (members, Uo) in enumerate(blk["basis"]):
        r = Uo.shape[1]
        if r:
            i0 = blk["orb_off"][o]
            Hm[i0:i0 + r * nb] = project_slab(P, blk, o, orbit_slab(P, members, mx_all))
        if log:
            log(o)
    return Hm


def project_vector(P, blk, B):
    """B_mu = U_mu^T B orbit by orbit (the same per-orbit bases)."""
    nb = P["nv"] * P["nc"]
    Bk = np.asarray(B).reshape(P["nk"], nb)
    out = np.zeros(blk["n"], dtype=np.result_type(B, np.float64))
    for o, (members, Uo) in enumerate(blk["basis"]):
        r = Uo.shape[1]
        if r:
            i0 = blk["orb_off"][o]
            out[i0:i0 + r * nb] = (Uo.T @ Bk[members]).reshape(-1)
    return out


def dipole_active(P, tol=1e-12):
    """Irreps whose projected dipole carries weight (Sec. III.D.1)."""
    nb2 = np.sum(np.abs(P["B"]) ** 2)
    act = []
    for nm, d, chi in P["group"]["irreps"]:
        blk = isotypic_basis(P, nm)
        if blk["n"] == 0:
            continue
        Bm = basis_matrix(P, blk).T @ P["B"]
        if np.sum(np.abs(Bm) ** 2) > tol * nb2:
            act.append(nm)
    return act


# ----------------------------------------------------------------------------
# eigenpairs, oscillator strengths and eps2
# ----------------------------------------------------------------------------
def eigh(H):
    return np.linalg.eigh(H)


def clusters(w, rel=1e-9):
    """Group ascending eigenvalues whose gaps are below rel*max(1,|w|)."""
    starts = [0]
    for i in range(1, len(w)):
        if w[i] - w[i - 1] > rel * max(1.0, abs(w[i])):
            starts.append(i)
    return starts + [len(w)]


def oscillator_strengths(w, A, B):
    """|B_l|^2 = |A_l^dag B|^2 summed within degenerate clusters.

    Returns (cluster energies, cluster weights, cluster sizes).
    """
    b = np.abs(A.conj().T @ B) ** 2
    st = clusters(w)
    e = np.array([w[st[i]:st[i + 1]].mean() for i in range(len(st) - 1)])
    s = np.array([b[st[i]:st[i + 1]].sum() for i in range(len(st) - 1)])
    m = np.array([st[i + 1] - st[i] for i in range(len(st) - 1)])
    return e, s, m


def eps2(omega_l, weight_l, nk, eta, wgrid):
    """(8 pi / N_k) sum_l |B_l|^2 [L(w - W_l) + L(w + W_l)]."""
    x1 = wgrid[:, None] - omega_l[None, :]
    x2 = wgrid[:, None] + omega_l[None, :]
    L = eta / (x1 * x1 + eta * eta) + eta / (x2 * x2 + eta * eta)
    return (8 * np.pi / nk) * (L @ weight_l)


def solve_block(P, irrep_name, H=None, nlow=100):
    """Oracle pipeline for one irrep block: H_mu, its spectrum, weights, eps2."""
    if H is None:
        H = hamiltonian(P)
    blk = isotypic_basis(P, irrep_name)
    U = basis_matrix(P, blk)
    Hm = project(H, U)
    Bm = U.T @ P["B"]
    w, A = eigh(Hm)
    e, s, m = oscillator_strengths(w, A, Bm)
    return dict(blk=blk, Hmu=Hm, Bmu=Bm, omega=w, A=A, cl_e=e, cl_w=s, cl_m=m,
                lowest=w[:nlow])


# ----------------------------------------------------------------------------
# longitudinal excitons, Sec. III.D.2: adding the G = 0 Coulomb term
# c B B^dag (c = 4 pi / (N_k V), times the spin factor 2 of the exchange, as in
# eps2) to the block leaves dark directions unchanged and moves each weighted
# pole to a root of the secular equation, Eq. (secular),
#     f(x) = 1 - c sum_i w_i / (x - p_i) = 0,
# one root between consecutive weighted poles and one above the highest.  The
# eigenvector components of Eq. (eigenvec_xi) give the new strengths
#     w'_xi = (B^T A')^2 / |A'|^2 = 1 / (c^2 sum_i w_i / (x_xi - p_i)^2).
# ----------------------------------------------------------------------------
def secular_roots(poles, weights, c, iters=200):
    """Roots of Eq. (secular) for the weighted poles (ascending, w > 0) by
    bisection in every interval at once."""
    p = np.asarray(poles, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    m = len(p)
    lo = p.copy()
    hi = np.append(p[1:], p[-1] + c * w.sum())

    def f(x):
        return 1.0 - c * np.sum(w[None, :] / (x[:, None] - p[None, :]), axis=1)

    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        neg = f(mid) < 0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    x = 0.5 * (lo + hi)
    assert len(x) == m
    return x


def secular_weights(roots, poles, weights, c):
    """Strengths of the longitudinal excitons from Eq. (eigenvec_xi)."""
    d = np.asarray(roots)[:, None] - np.asarray(poles)[None, :]
    return 1.0 / (c * c * np.sum(np.asarray(weights)[None, :] / d ** 2, axis=1))


def eels(cl_e, cl_w, nk, rel=1e-14):
    """Longitudinal poles and strengths from the clustered optical poles."""
    keep = cl_w > rel * cl_w.sum()
    p, w = cl_e[keep], cl_w[keep]
    c = 8.0 * np.pi / nk
    x = secular_roots(p, w, c)
    return x, secular_weights(x, p, w, c)


# ----------------------------------------------------------------------------
# Lanczos-Haydock per block (the alternative to diagonalisation that the
# block structure also serves, Sec. III.D.1): Lanczos on H_mu started from
# v_0 = B_mu / |B_mu| gives the tridiagonal coefficients a_j, b_j; the
# resolvent element v_0^dag (z - H_mu)^-1 v_0 is the continued fraction
#     G(z) = 1 / (z - a_0 - b_1^2 / (z - a_1 - b_2^2 / (...)))
# truncated after K levels, and since L_eta(x) = -Im 1/(x + i eta),
#     eps2(w) = (8 pi / N_k) |B_mu|^2 (-Im G(w + i eta) - Im G(-w + i eta)),
# the same two terms as in eps2 above.
# ----------------------------------------------------------------------------
def haydock_coefficients(Hm, Bm, K):
    """Plain Lanczos (no reorthogonalisation): a[0..K'), b[0..K'] with
    b[0] = |B_mu| and b[j] (j >= 1) the norm of the j-th residual; stops early
    (K' < K) when a residual vanishes (the Krylov space is invariant)."""
    Hm = np.asarray(Hm, dtype=np.complex128)
    v = np.asarray(Bm, dtype=np.complex128)
    bn = np.linalg.norm(v)
    a, b = [], [bn]
    v_prev = np.zeros_like(v)
    v = v / bn
    beta = 0.0
    for j in range(K):
        w = Hm @ v - beta * v_prev
        alpha = float(np.real(np.vdot(v, w)))
        w = w - alpha * v
        beta = float(np.linalg.norm(w))
        a.append(alpha)
        b.append(beta)
        if beta == 0.0:
            break
        v_prev, v = v, w / beta
    return np.array(a), np.array(b)


def continued_fraction(a, b, z):
    """G(z) for the coefficients of haydock_coefficients, evaluated from the
    deepest level up (the remainder below level K is dropped)."""
    z = np.asarray(z, dtype=np.complex128)
    g = np.zeros_like(z)
    for j in range(len(a) - 1, -1, -1):
        tail = b[j + 1] ** 2 * g if j + 1 < len(a) else 0.0
        g = 1.0 / (z - a[j] - tail)
    return g


def haydock_eps2(a, b, nk, eta, wgrid):
    w = np.asarray(wgrid, dtype=np.float64)
    g1 = continued_fraction(a, b, w + 1j * eta)
    g2 = continued_fraction(a, b, -w + 1j * eta)
    return (8 * np.pi / nk) * b[0] ** 2 * (-g1.imag - g2.imag)
