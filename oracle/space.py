"""Global conforming displacement space on a structured mixed-p quad mesh.

Test infrastructure only (see the package docstring).

Each element e = ey*nelx + ex carries its own order p_e (Sec. 3: the dp-mesh
has per-element p).  The paper requires a compatible mixed-p field but does
not spell out the construction; the reading used here is the conforming H1
space of continuous fields that are Q_{p_e} on every element, i.e. the
'minimum rule': a shared edge carries the edge modes k = 2..min(p_a, p_b),
a boundary edge carries k = 2..p_e, and edge modes of the higher-order
neighbour above the edge degree are absent.  With the hierarchic basis of
``fem.basis_1d`` an edge mode k has the same trace phi_k on both sides (all
elements share one orientation), so no sign changes are needed.

Global scalar numbering (vector DOF = 2*id + component):
  1. vertices            id = vy*(nelx+1) + vx
  2. horizontal edges    edge index vy*nelx + ex, each a block of modes 2..deg
  3. vertical edges      edge index ey*(nelx+1) + vx, each a block of modes
  4. element interiors   per element in order e, modes (i, j) with i, j >= 2,
                         i fastest
"""

from dataclasses import dataclass

import numpy as np

SUP_VERTEX, SUP_EDGE_LEFT, SUP_EDGE_RIGHT, SUP_EDGE_BOTTOM, SUP_EDGE_TOP = 0, 1, 2, 3, 4


@dataclass
class DofSpace:
    nelx: int
    nely: int
    p: np.ndarray          # [nel] int
    n_scalar: int          # number of scalar ids
    n_dof: int             # 2 * n_scalar
    hdeg: np.ndarray       # [nelx*(nely+1)] degree of each horizontal edge
    vdeg: np.ndarray       # [(nelx+1)*nely]
    hoff: np.ndarray       # first scalar id of each horizontal edge block
    voff: np.ndarray
    ioff: np.ndarray       # first scalar id of each element's interior block
    n_vertex: int


def build_space(nelx, nely, p):
    """Numbers the conforming mixed-p space described in the module docstring."""
    p = np.asarray(p, dtype=np.int64).reshape(nely, nelx)
    nv = (nelx + 1) * (nely + 1)
    # Horizontal edge (ex, vy): elements (ex, vy-1) below and (ex, vy) above.
    hdeg = np.zeros((nely + 1, nelx), dtype=np.int64)
    for vy in range(nely + 1):
        for ex in range(nelx):
            adj = []
            if vy > 0:
                adj.append(p[vy - 1, ex])
            if vy < nely:
                adj.append(p[vy, ex])
            hdeg[vy, ex] = min(adj)
    # Vertical edge (vx, ey): elements (vx-1, ey) left and (vx, ey) right.
    vdeg = np.zeros((nely, nelx + 1), dtype=np.int64)
    for ey in range(nely):
        for vx in range(nelx + 1):
            adj = []
            if vx > 0:
                adj.append(p[ey, vx - 1])
            if vx < nelx:
                adj.append(p[ey, vx])
            vdeg[ey, vx] = min(adj)
    hdeg = hdeg.ravel()
    vdeg = vdeg.ravel()
    nmode_h = np.maximum(hdeg - 1, 0)
    nmode_v = np.maximum(vdeg - 1, 0)
    hoff = nv + np.concatenate([[0], np.cumsum(nmode_h)[:-1]])
    nh_total = int(nmode_h.sum())
    voff = nv + nh_total + np.concatenate([[0], np.cumsum(nmode_v)[:-1]])
    nvert_total = int(nmode_v.sum())
    nint = (p.ravel() - 1) ** 2
    ioff = nv + nh_total + nvert_total + np.concatenate([[0], np.cumsum(nint)[:-1]])
    n_scalar = nv + nh_total + nvert_total + int(nint.sum())
    return DofSpace(nelx, nely, p.ravel().copy(), n_scalar, 2 * n_scalar, hdeg, vdeg,
                    hoff.astype(np.int64), voff.astype(np.int64), ioff.astype(np.int64), nv)


def element_scalar_ids(space, e):
    """Global scalar id of each local function (i, j) of element e, indexed
    by the local scalar number a = j (p+1) + i; -1 where the function is not
    part of the conforming space (an edge mode above the edge degree)."""
    nelx = space.nelx
    ex, ey = e % nelx, e // nelx
    pe = int(space.p[e])
    n1 = pe + 1
    ids = np.full(n1 * n1, -1, dtype=np.int64)
    for j in range(n1):
        for i in range(n1):
            a = j * n1 + i
            if i <= 1 and j <= 1:
                ids[a] = (ey + j) * (nelx + 1) + (ex + i)
            elif j <= 1:  # i >= 2: mode i on horizontal edge (ex, ey + j)
                h = (ey + j) * nelx + ex
                if i <= space.hdeg[h]:
                    ids[a] = space.hoff[h] + (i - 2)
            elif i <= 1:  # j >= 2: mode j on vertical edge (ex + i, ey)
                v = ey * (nelx + 1) + ex + i
                if j <= space.vdeg[v]:
                    ids[a] = space.voff[v] + (j - 2)
            else:
                ids[a] = space.ioff[e] + (j - 2) * (pe - 1) + (i - 2)
    return ids


def fixed_scalar_ids(space, supports):
    """Scalar ids fixed in each component by the supports.

    A support is (kind, a, b, comp_mask), comp_mask bit 0 = x, bit 1 = y.
    An edge support fixes the component on every vertex of that boundary and
    on every edge mode of its edges (so the whole trace is zero); a vertex
    support (kind 0, vertex (a, b)) fixes the vertex function only.
    Returns two sets (x-fixed ids, y-fixed ids)."""
    nelx, nely = space.nelx, space.nely
    fixed = (set(), set())
    for kind, a, b, mask in supports:
        ids = []
        if kind == SUP_VERTEX:
            ids.append(b * (nelx + 1) + a)
        elif kind in (SUP_EDGE_LEFT, SUP_EDGE_RIGHT):
            vx = 0 if kind == SUP_EDGE_LEFT else nelx
            for vy in range(nely + 1):
                ids.append(vy * (nelx + 1) + vx)
            for ey in range(nely):
                v = ey * (nelx + 1) + vx
                ids.extend(range(space.voff[v], space.voff[v] + max(space.vdeg[v] - 1, 0)))
        elif kind in (SUP_EDGE_BOTTOM, SUP_EDGE_TOP):
            vy = 0 if kind == SUP_EDGE_BOTTOM else nely
            for vx in range(nelx + 1):
                ids.append(vy * (nelx + 1) + vx)
            for ex in range(nelx):
                h = vy * nelx + ex
                ids.extend(range(space.hoff[h], space.hoff[h] + max(space.hdeg[h] - 1, 0)))
        else:
            raise ValueError(f"unknown support kind {kind}")
        for c in range(2):
            if mask & (1 << c):
                fixed[c].update(int(i) for i in ids)
    return fixed
