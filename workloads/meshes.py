"""Mesh generators and integer trace maps.

Element node conventions (shared by both sides as *data*):

* quad / hex: reference element [-1, 1]^d, nodes on a tensor lattice with
  multi-index (i, j[, k]) in 0..p, ordered with i (x) fastest.  Reference
  vertices are the 2^d corners in the same lexicographic order.  Local faces:
  xi=-1, xi=+1, eta=-1, eta=+1, zeta=-1, zeta=+1.
* tri / tet: reference simplex with vertices 0, e_x, e_y[, e_z]; equispaced
  nodes with multi-index (i, j[, k]), i + j (+ k) <= p, ordered k outer,
  j middle, i inner.  Local face f is the face opposite vertex f.
* Face node b of local face f is the b-th element node (ascending element node
  index) lying on that face.

Trace maps take (element, local face, face node) to a global trace node.  HDG
gives each mesh face its own nodes, EDG shares every skeleton lattice point,
IEDG shares on interior faces and keeps boundary faces private (the paper's
section on examples of schemes within the hybridized DG family).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

ETYPE_CODE = {"tri": 0, "quad": 1, "tet": 2, "hex": 3}
ETYPE_DIM = {"tri": 2, "quad": 2, "tet": 3, "hex": 3}
ETYPE_NV = {"tri": 3, "quad": 4, "tet": 4, "hex": 8}
ETYPE_NF = {"tri": 3, "quad": 4, "tet": 4, "hex": 6}


# ----------------------------------------------------------------------------
# node lattices (integer data only)
# ----------------------------------------------------------------------------
def node_multi_indices(etype: str, p: int) -> np.ndarray:
    """Integer multi-indices of the element nodes in element node order."""
    d = ETYPE_DIM[etype]
    out = []
    if etype in ("quad", "hex"):
        rng = range(p + 1)
        if d == 2:
            for j in rng:
                for i in rng:
                    out.append((i, j))
        else:
            for k in rng:
                for j in rng:
                    for i in rng:
                        out.append((i, j, k))
    else:
        if d == 2:
            for j in range(p + 1):
                for i in range(p + 1 - j):
                    out.append((i, j))
        else:
            for k in range(p + 1):
                for j in range(p + 1 - k):
                    for i in range(p + 1 - j - k):
                        out.append((i, j, k))
    return np.array(out, dtype=np.int64)


def face_nodes(etype: str, p: int) -> list[np.ndarray]:
    """For each local face, the element node indices on it (ascending)."""
    mi = node_multi_indices(etype, p)
    faces = []
    if etype in ("quad", "hex"):
        d = ETYPE_DIM[etype]
        for f in range(2 * d):
            axis, side = divmod(f, 2)
            val = 0 if side == 0 else p
            faces.append(np.nonzero(mi[:, axis] == val)[0])
    else:
        tot = mi.sum(axis=1)
        d = ETYPE_DIM[etype]
        faces.append(np.nonzero(tot == p)[0])          # opposite vertex 0
        for f in range(1, d + 1):                      # opposite vertex f
            faces.append(np.nonzero(mi[:, f - 1] == 0)[0])
    return faces


def n_face_nodes(etype: str, p: int) -> int:
    return len(face_nodes(etype, p)[0])


def n_nodes(etype: str, p: int) -> int:
    return len(node_multi_indices(etype, p))


# ----------------------------------------------------------------------------
# mesh container
# ----------------------------------------------------------------------------
@dataclass
class Mesh:
    etype: str
    elem_xyz: np.ndarray          # (E, nv, d) float64 vertex coordinates
    elem_lat: np.ndarray          # (E, nv, d) int64 unjittered lattice coords
    period: np.ndarray | None     # (d,) lattice period (cells) or None
    boundary: np.ndarray          # (E, nf) bool, face on the domain boundary
    h: float                      # cell size
    extent: np.ndarray            # (d,) domain lower corner
    length: np.ndarray            # (d,) domain edge lengths
    info: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return ETYPE_DIM[self.etype]

    @property
    def n_elem(self) -> int:
        return self.elem_xyz.shape[0]

    @property
    def nf(self) -> int:
        return ETYPE_NF[self.etype]

    def subset(self, idx) -> "Mesh":
        idx = np.asarray(idx)
        return Mesh(self.etype, self.elem_xyz[idx].copy(), self.elem_lat[idx].copy(), self.period,
                    self.boundary[idx].copy(), self.h, self.extent, self.length, dict(self.info))


def _jitter(rng, shape_lattice, d, amp, periodic, n_cells):
    """Per-lattice-vertex displacement U(-amp, amp)^d; boundary fixed if not periodic."""
    disp = rng.uniform(-amp, amp, size=tuple(shape_lattice) + (d,))
    if not periodic:
        for ax in range(d):
            sl = [slice(None)] * d
            sl[ax] = 0
            disp[tuple(sl)] = 0.0
            sl[ax] = n_cells
            disp[tuple(sl)] = 0.0
    return disp


def _vertex_xyz(lat, disp, periodic, n_cells, h, lo):
    """Coordinates of integer lattice vertices (E, nv, d) with periodic unwrapping."""
    d = lat.shape[-1]
    if periodic:
        wrapped = np.mod(lat, n_cells)
        dd = disp[tuple(wrapped[..., a] for a in range(d))]
    else:
        dd = disp[tuple(lat[..., a] for a in range(d))]
    return lo + lat * h + dd


def tri_square(n: int, jitter: float = 0.0, seed=0, periodic: bool = False,
               lo=0.0, length=1.0) -> Mesh:
    """[lo, lo+length]^2 split into n x n squares, each cut SW-NE into 2 triangles."""
    rng = np.random.default_rng(seed)
    h = length / n
    shape = (n, n) if periodic else (n + 1, n + 1)
    disp = _jitter(rng, shape, 2, jitter * h, periodic, n)
    lats = []
    for j in range(n):
        for i in range(n):
            sw, se, nw, ne = (i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)
            lats.append((sw, se, ne))   # counter-clockwise
            lats.append((sw, ne, nw))   # counter-clockwise
    lat = np.array(lats, dtype=np.int64)
    xyz = _vertex_xyz(lat, disp, periodic, n, h, lo)
    bnd = np.zeros((lat.shape[0], 3), dtype=bool)
    if not periodic:
        for e in range(lat.shape[0]):
            for f in range(3):
                vs = [lat[e, r] for r in range(3) if r != f]
                for ax in range(2):
                    if all(v[ax] == 0 for v in vs) or all(v[ax] == n for v in vs):
                        bnd[e, f] = True
    return Mesh("tri", xyz, lat, np.array([n, n]) if periodic else None, bnd, h,
                np.array([lo, lo], float), np.array([length, length], float),
                {"n": n, "jitter": jitter, "periodic": periodic})


def quad_square(n: int, jitter: float = 0.0, seed=0, periodic: bool = False,
                lo=0.0, length=1.0) -> Mesh:
    rng = np.random.default_rng(seed)
    h = length / n
    shape = (n, n) if periodic else (n + 1, n + 1)
    disp = _jitter(rng, shape, 2, jitter * h, periodic, n)
    lats = []
    for j in range(n):
        for i in range(n):
            lats.append([(i + a, j + b) for b in (0, 1) for a in (0, 1)])
    lat = np.array(lats, dtype=np.int64)
    xyz = _vertex_xyz(lat, disp, periodic, n, h, lo)
    bnd = np.zeros((lat.shape[0], 4), dtype=bool)
    if not periodic:
        for e in range(lat.shape[0]):
            i, j = lat[e, 0]
            bnd[e] = [i == 0, i == n - 1, j == 0, j == n - 1]
    return Mesh("quad", xyz, lat, np.array([n, n]) if periodic else None, bnd, h,
                np.array([lo, lo], float), np.array([length, length], float),
                {"n": n, "jitter": jitter, "periodic": periodic})


def hex_cube(n: int, jitter: float = 0.0, seed=0, periodic: bool = True,
             lo=0.0, length=2 * np.pi) -> Mesh:
    """[lo, lo+length]^3 in n^3 trilinear hexahedra with seeded vertex jitter."""
    rng = np.random.default_rng(seed)
    h = length / n
    shape = (n, n, n) if periodic else (n + 1, n + 1, n + 1)
    disp = _jitter(rng, shape, 3, jitter * h, periodic, n)
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                     kk.transpose(2, 1, 0).ravel()], axis=1)  # element order: i fastest
    corners = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.int64)
    lat = base[:, None, :] + corners[None, :, :]
    xyz = _vertex_xyz(lat, disp, periodic, n, h, lo)
    bnd = np.zeros((lat.shape[0], 6), dtype=bool)
    if not periodic:
        b0 = lat[:, 0, :]
        for ax in range(3):
            bnd[:, 2 * ax] = b0[:, ax] == 0
            bnd[:, 2 * ax + 1] = b0[:, ax] == n - 1
    return Mesh("hex", xyz, lat, np.array([n, n, n]) if periodic else None, bnd, h,
                np.full(3, lo, float), np.full(3, length, float),
                {"n": n, "jitter": jitter, "periodic": periodic})


def kuhn_tets(n: int, jitter: float = 0.0, seed=0, periodic: bool = True,
              lo=0.0, length=2 * np.pi) -> Mesh:
    """n^3 cubes, each split into 6 tetrahedra along its main diagonal (Kuhn / Freudenthal)."""
    rng = np.random.default_rng(seed)
    h = length / n
    shape = (n, n, n) if periodic else (n + 1, n + 1, n + 1)
    disp = _jitter(rng, shape, 3, jitter * h, periodic, n)
    eye = np.eye(3, dtype=np.int64)
    lats = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                o = np.array([i, j, k], dtype=np.int64)
                for perm in itertools.permutations(range(3)):
                    v0 = o
                    v1 = v0 + eye[perm[0]]
                    v2 = v1 + eye[perm[1]]
                    v3 = v2 + eye[perm[2]]
                    vs = [v0, v1, v2, v3]
                    det = np.linalg.det(np.stack([v1 - v0, v2 - v0, v3 - v0]).astype(float))
                    if det < 0:
                        vs = [v0, v2, v1, v3]
                    lats.append(vs)
    lat = np.array(lats, dtype=np.int64)
    xyz = _vertex_xyz(lat, disp, periodic, n, h, lo)
    bnd = np.zeros((lat.shape[0], 4), dtype=bool)
    if not periodic:
        for e in range(lat.shape[0]):
            for f in range(4):
                vs = np.array([lat[e, r] for r in range(4) if r != f])
                for ax in range(3):
                    if np.all(vs[:, ax] == 0) or np.all(vs[:, ax] == n):
                        bnd[e, f] = True
    return Mesh("tet", xyz, lat, np.array([n, n, n]) if periodic else None, bnd, h,
                np.full(3, lo, float), np.full(3, length, float),
                {"n": n, "jitter": jitter, "periodic": periodic})


# ----------------------------------------------------------------------------
# trace maps
# ----------------------------------------------------------------------------
def node_lattice_keys(mesh: Mesh, p: int) -> np.ndarray:
    """Integer key of every element node on the p-refined lattice, (E, Np, d).

    Periodic dimensions are reduced modulo n*p so that identified points agree.
    """
    mi = node_multi_indices(mesh.etype, p)          # (Np, d)
    lat = mesh.elem_lat
    if mesh.etype in ("quad", "hex"):
        keys = p * lat[:, 0, None, :] + mi[None, :, :]
    else:
        v0 = lat[:, 0, :]
        keys = p * v0[:, None, :].copy()
        for r in range(mi.shape[1]):
            keys = keys + mi[None, :, r, None] * (lat[:, r + 1, None, :] - v0[:, None, :])
    if mesh.period is not None:
        keys = np.mod(keys, mesh.period * p)
    return keys


def _encode(keys: np.ndarray, base: int) -> np.ndarray:
    """Encode integer d-vectors (non-negative, < base) into int64 scalars."""
    out = np.zeros(keys.shape[:-1], dtype=np.int64)
    for a in range(keys.shape[-1]):
        out = out * base + keys[..., a]
    return out


def trace_map(mesh: Mesh, p: int, scheme: str = "hdg"):
    """Global trace node of every (element, local face, face node).

    Returns (tmap (E, nf, Nfp) int32, n_trace).  ``scheme`` is 'hdg', 'edg' or
    'iedg'.
    """
    scheme = scheme.lower()
    if mesh.period is not None and np.any(mesh.period * p < 3):
        raise ValueError("periodic lattice too small to identify faces: need n*p >= 3")
    fn = face_nodes(mesh.etype, p)
    nfp = len(fn[0])
    keys = node_lattice_keys(mesh, p)
    base = int(keys.max()) + 2
    code = _encode(keys, base)                           # (E, Np)
    E, nf = mesh.n_elem, mesh.nf
    fcode = np.stack([code[:, fn[f]] for f in range(nf)], axis=1)   # (E, nf, Nfp)
    tmap = np.empty((E, nf, nfp), dtype=np.int64)

    # faces: identify by the sorted tuple of node codes
    fsorted = np.sort(fcode, axis=2)
    flat = fsorted.reshape(E * nf, nfp)
    _, face_id, face_count = np.unique(flat, axis=0, return_inverse=True, return_counts=True)
    face_id = face_id.reshape(E, nf)
    if np.any(face_count > 2):
        raise ValueError("non-conforming mesh: a face is shared by more than two elements")
    # position of each face node within the canonical (sorted) order of its face
    order = np.argsort(fcode, axis=2, kind="stable")
    pos = np.empty_like(order)
    np.put_along_axis(pos, order, np.arange(nfp)[None, None, :].repeat(E, 0).repeat(nf, 1), axis=2)

    if scheme == "hdg":
        tmap = face_id[:, :, None] * nfp + pos
        n_trace = int(face_id.max() + 1) * nfp
    elif scheme in ("edg", "iedg"):
        shared = np.ones((E, nf), dtype=bool)
        if scheme == "iedg":
            shared = ~mesh.boundary
        uniq, inv = np.unique(fcode[shared], return_inverse=True)
        tm_shared = inv
        n_sh = len(uniq)
        tmap = np.empty((E, nf, nfp), dtype=np.int64)
        tmap[shared] = tm_shared.reshape(-1, nfp)
        if scheme == "iedg" and np.any(~shared):
            bid = face_id[~shared]
            _, binv = np.unique(bid, return_inverse=True)
            tmap[~shared] = n_sh + binv[:, None] * nfp + pos[~shared]
            n_trace = n_sh + (int(binv.max()) + 1) * nfp
        else:
            n_trace = n_sh
    else:
        raise ValueError(scheme)
    return tmap.astype(np.int32), int(n_trace)


def face_neighbors(mesh: Mesh, p: int = 1):
    """(E, nf) neighbour element across each face (-1 on the boundary) and its local face."""
    fn = face_nodes(mesh.etype, p)
    keys = node_lattice_keys(mesh, p)
    base = int(keys.max()) + 2
    code = _encode(keys, base)
    E, nf = mesh.n_elem, mesh.nf
    fcode = np.sort(np.stack([code[:, fn[f]] for f in range(nf)], axis=1), axis=2)
    flat = fcode.reshape(E * nf, -1)
    _, fid = np.unique(flat, axis=0, return_inverse=True)
    fid = fid.reshape(-1)
    nb = -np.ones((E * nf,), dtype=np.int64)
    nbf = -np.ones((E * nf,), dtype=np.int64)
    order = np.argsort(fid, kind="stable")
    sf = fid[order]
    same = np.nonzero(sf[1:] == sf[:-1])[0]
    a, b = order[same], order[same + 1]
    nb[a], nbf[a] = b // nf, b % nf
    nb[b], nbf[b] = a // nf, a % nf
    return nb.reshape(E, nf), nbf.reshape(E, nf)


def subset_mesh(mesh: Mesh, elems) -> Mesh:
    """The elements `elems` of `mesh` as a mesh of their own.

    Faces whose neighbour is not in the subset become boundary faces; the
    lattice period is kept, so faces matched across a periodic boundary stay
    matched.
    """
    elems = np.asarray(elems, dtype=np.int64)
    nb, _ = face_neighbors(mesh)
    inside = np.zeros(mesh.n_elem, dtype=bool)
    inside[elems] = True
    nbs = nb[elems]
    bnd = mesh.boundary[elems] | (nbs < 0) | ~inside[np.maximum(nbs, 0)]
    return Mesh(mesh.etype, mesh.elem_xyz[elems].copy(), mesh.elem_lat[elems].copy(), mesh.period, bnd, mesh.h,
                mesh.extent, mesh.length, dict(mesh.info, subset=len(elems)))
