"""Point groups Oh and D6h: operations, classes and character tables.

Paper: Sec. III.C.1 (a symmetry operation acts on k by a rotation matrix and a
fold back into the Brillouin zone, Eq. (sk)); Sec. III.C.4 (the characters of
the irreps are all that the projectors need, Eq. (LOT), Eq. (projection)).
Only linear operations are used (no time reversal), as in Sec. III.C.3.

Each group is returned as a dict with
  kmat[nops,3,3]  integer matrix acting on reduced k coordinates,
  rcart[nops,3,3] Cartesian matrix (acts on dipole vectors),
  irreps          list of (name, dim, chi[nops]) with real characters.
"""
import itertools
import math
import numpy as np

# Character table of O (proper rotations), columns E, C3, C2 (=C4^2), C4, C2'.
_O_TABLE = {
    "A1": (1, [1, 1, 1, 1, 1]),
    "A2": (1, [1, 1, 1, -1, -1]),
    "E": (2, [2, -1, 2, 0, 0]),
    "T1": (3, [3, 0, -1, 1, -1]),
    "T2": (3, [3, 0, -1, -1, 1]),
}
_O_CLASSES = ["E", "C3", "C2", "C4", "C2p"]

# Character table of D6, columns E, C6, C3, C2, C2' (axes along a1, a2, a1+a2), C2''.
_D6_TABLE = {
    "A1": (1, [1, 1, 1, 1, 1, 1]),
    "A2": (1, [1, 1, 1, 1, -1, -1]),
    "B1": (1, [1, -1, 1, -1, 1, -1]),
    "B2": (1, [1, -1, 1, -1, -1, 1]),
    "E1": (2, [2, 1, -1, -2, 0, 0]),
    "E2": (2, [2, -1, -1, 2, 0, 0]),
}
_D6_CLASSES = ["E", "C6", "C3", "C2", "C2p", "C2pp"]


def _oh_class(R):
    """Class in O of the proper part det(R) R of a signed permutation matrix."""
    P = int(round(np.linalg.det(R))) * R
    t = int(np.trace(P))
    if t == 3:
        return "E"
    if t == 0:
        return "C3"
    if t == 1:
        return "C4"
    assert t == -1
    return "C2" if np.count_nonzero(P - np.diag(np.diag(P))) == 0 else "C2p"


def group_oh():
    """The 48 signed 3x3 permutation matrices (full cubic group m-3m)."""
    ops = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            ops.append(R)
    ops = np.array(ops)
    det = np.array([int(round(np.linalg.det(R))) for R in ops])
    cls = [_oh_class(R) for R in ops]
    irreps = []
    for par, sgn in (("g", 1), ("u", -1)):
        for name, (d, row) in _O_TABLE.items():
            chi = np.array([row[_O_CLASSES.index(c)] * (1 if sgn == 1 else det[s])
                            for s, c in enumerate(cls)], dtype=np.float64)
            irreps.append((name + par, d, chi))
    return dict(name="Oh", lattice="cubic", kmat=ops, rcart=ops.astype(np.float64),
                irreps=irreps, classes=cls)


def _rot(axis_angle, theta):
    """3x3 rotation by theta about the unit vector axis_angle (z or in-plane)."""
    if axis_angle is None:  # about z
        c, s = math.cos(theta), math.sin(theta)
        return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    ax = np.array([math.cos(axis_angle), math.sin(axis_angle), 0.0])
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + math.sin(theta) * K + (1 - math.cos(theta)) * (K @ K)


def group_d6h():
    """D6h (6/mmm) for a hexagonal lattice a1=(1,0), a2=(-1/2, sqrt3/2).

    Reduced reciprocal basis b1 = (1, 1/sqrt3), b2 = (0, 2/sqrt3) (times 2pi/a);
    k-action matrices are B^-1 R B with B = [b1 b2], extended by R_zz on k3.
    """
    proper, cls = [], []
    for m in range(6):
        proper.append(_rot(None, m * math.pi / 3))
        cls.append(["E", "C6", "C3", "C2", "C3", "C6"][m])
    for j in range(6):  # in-plane two-fold axes every 30 degrees
        proper.append(_rot(j * math.pi / 6, math.pi))
        cls.append("C2p" if j % 2 == 0 else "C2pp")  # 0, 60, 120 deg: along a1, a1+a2, a2
    rc = proper + [-R for R in proper]
    cls = cls + cls
    det = [1] * 12 + [-1] * 12
    B = np.array([[1.0, 0.0], [1 / math.sqrt(3), 2 / math.sqrt(3)]])
    kmat = []
    for R in rc:
        M2 = np.linalg.solve(B, R[:2, :2] @ B)
        Mi = np.rint(M2).astype(np.int64)
        assert np.abs(M2 - Mi).max() < 1e-9
        M = np.zeros((3, 3), dtype=np.int64)
        M[:2, :2] = Mi
        M[2, 2] = int(round(R[2, 2]))
        kmat.append(M)
    irreps = []
    for par, sgn in (("g", 1), ("u", -1)):
        for name, (d, row) in _D6_TABLE.items():
            chi = np.array([row[_D6_CLASSES.index(c)] * (1 if sgn == 1 else det[s])
                            for s, c in enumerate(cls)], dtype=np.float64)
            irreps.append((name + par, d, chi))
    return dict(name="D6h", lattice="hex", kmat=np.array(kmat), rcart=np.array(rc),
                irreps=irreps, classes=cls)


def group(name):
    return {"Oh": group_oh, "D6h": group_d6h}[name]()


def irrep(g, name):
    for nm, d, chi in g["irreps"]:
        if nm == name:
            return d, chi
    raise KeyError(name)


def multiplication_table(kmat):
    """table[a, b] = index of kmat[a] @ kmat[b] (checks closure)."""
    idx = {m.tobytes(): i for i, m in enumerate(kmat)}
    n = len(kmat)
    t = np.empty((n, n), dtype=np.int64)
    for a in range(n):
        for b in range(n):
            t[a, b] = idx[(kmat[a] @ kmat[b]).tobytes()]
    return t
