"""Assembled-matrix reference solve: K u = f, compliance and sensitivities.

Test infrastructure only (see the package docstring).

Follows Sec. 2.2: the global K is the assembly of element matrices K_e, each
the sum over density cells of E(rho_{e,s}) K_s (composite integration of
Appendix B with the SIMP law of Sec. 2.2); u solves K u = f (Eq.
``eq_comp_1``) with the supported DOFs eliminated; the objective is
J = z^T u with z = f (Sec. 4.1), i.e. the compliance.

Solve: a sparse LU factorisation (SuperLU, symmetric ordering, no pivoting
since K_ff is symmetric positive definite) of the free-free block, then
iterative refinement with the residual r = f - K u accumulated in
numpy.longdouble, until the correction is below 1e-15 of u.  (With modulus
contrast E_min/E0 = 1e-9 the condition number of K is large, so a single
FP64 factor solve alone is not trusted to 1e-8.)

The residual applies K by its definition, element by element:
K u = sum_e P_e^T K_e (u_e - r_e), where r_e is the rigid motion that takes
the element's values at three vertex DOFs (vertex (0,0) x and y, vertex
(1,0) y).  K_e annihilates rigid motions, so this is K u exactly; it matters
in floating point.  Where a region of solid material is joined to the
supports only through void material (E = E_min), the region moves almost
rigidly by 1e9 times its deformation.  The FP64 cell matrices annihilate
rigid motions only to their rounding (K_s r ~ 1e-16 |K_s| |r|), and the
assembled FP64 matrix only to the rounding of its sums, so applying them to
the whole of u_e puts spurious forces of 1e-7 relative size on such a
region, which move u by up to 1e-3.  Applied to u_e - r_e they act on the
deformation alone.  The assembled FP64 matrix serves only as the
preconditioner of the refinement (its LU factors).

Sensitivity: for the self-adjoint compliance the adjoint is lambda = -u, so
dc/drho_{e,s} = -u^T (dK/drho_{e,s}) u = -E'(rho_{e,s}) u_e^T K_s u_e,
evaluated as (u_e - r_e)^T K_s (u_e - r_e) for the same reason.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import subcell_stiffness, simp_modulus, simp_modulus_derivative
from .space import build_space, element_scalar_ids, fixed_scalar_ids


def element_dofs_global(space, e):
    """Global vector DOF of each local DOF 2a + c of element e (-1: absent)."""
    ids = element_scalar_ids(space, e)
    out = np.full(2 * ids.size, -1, dtype=np.int64)
    ok = ids >= 0
    out[0::2][ok] = 2 * ids[ok]
    out[1::2][ok] = 2 * ids[ok] + 1
    return out


def cell_offsets(d):
    """Start of each element's density cells in the element-major density
    vector (cell order sy*d + sx within an element)."""
    d = np.asarray(d, dtype=np.int64)
    return np.concatenate([[0], np.cumsum(d * d)])


def assemble(nelx, nely, p, d, rho, E0, Emin, q, nu, ks_cache=None):
    """Assembled global stiffness K (all DOFs, CSR), the space and per-element
    data.  K = sum_e P_e^T (sum_s E(rho_{e,s}) K_s) P_e."""
    p = np.asarray(p, dtype=np.int64).ravel()
    d = np.asarray(d, dtype=np.int64).ravel()
    rho = np.asarray(rho, dtype=np.float64).ravel()
    nel = nelx * nely
    assert p.size == nel and d.size == nel
    off = cell_offsets(d)
    assert rho.size == off[-1]
    space = build_space(nelx, nely, p)
    if ks_cache is None:
        ks_cache = {}
    E = simp_modulus(rho, E0, Emin, q)
    rows, cols, vals = [], [], []
    edofs = [element_dofs_global(space, e) for e in range(nel)]
    for (pe, de) in sorted(set(zip(p.tolist(), d.tolist()))):
        key = (pe, de, nu)
        if key not in ks_cache:
            ks_cache[key] = subcell_stiffness(pe, de, nu)
        Ks = ks_cache[key]
        S, ne, _ = Ks.shape
        els = np.nonzero((p == pe) & (d == de))[0]
        Eg = np.stack([E[off[e]:off[e] + S] for e in els])          # [n, S]
        Ke = (Eg @ Ks.reshape(S, ne * ne)).reshape(-1, ne, ne)       # [n, ne, ne]
        G = np.stack([edofs[e] for e in els])                        # [n, ne]
        valid = G >= 0
        for k, e in enumerate(els):
            m = valid[k]
            gi = G[k][m]
            blk = Ke[k][np.ix_(m, m)]
            rows.append(np.repeat(gi, gi.size))
            cols.append(np.tile(gi, gi.size))
            vals.append(blk.ravel())
    n = space.n_dof
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K, space, edofs, off, ks_cache


def load_vectors(space, loads, n_load_cases):
    """Point loads (vx, vy, fx, fy, load_case) at vertex DOFs."""
    f = np.zeros((n_load_cases, space.n_dof))
    for vx, vy, fx, fy, lc in loads:
        vid = vy * (space.nelx + 1) + vx
        f[lc, 2 * vid] += fx
        f[lc, 2 * vid + 1] += fy
    return f


def free_mask(space, supports):
    fx, fy = fixed_scalar_ids(space, supports)
    free = np.ones(space.n_dof, dtype=bool)
    for i in fx:
        free[2 * i] = False
    for i in fy:
        free[2 * i + 1] = False
    return free


def rigid_free(ue, p):
    """u_e minus the rigid motion (a - th y, b + th x) through its DOFs 0, 1
    (vertex (0,0) x, y) and 3 (vertex (1,0) y), for element vectors [..., n_e]
    of order p (the rigid motion lives on the four vertex functions)."""
    n1 = p + 1
    a, b = ue[..., 0], ue[..., 1]
    th = ue[..., 3] - ue[..., 1]
    out = ue.copy()
    for j in range(2):
        for i in range(2):
            k = j * n1 + i
            out[..., 2 * k] -= a - th * j
            out[..., 2 * k + 1] -= b + th * i
    return out


class ElementOperator:
    """K u = sum_e P_e^T K_e (u_e - r_e) in numpy.longdouble, element group
    by element group, with K_e = sum_s E(rho_{e,s}) K_s (Sec. 2.2, Appendix
    B) and r_e the element's rigid motion (rigid_free)."""

    def __init__(self, p, d, E, edofs, off, ks, nu, n_dof):
        p = np.asarray(p, dtype=np.int64).ravel()
        d = np.asarray(d, dtype=np.int64).ravel()
        self.n_dof = n_dof
        self.groups = []
        for (pe, de) in sorted(set(zip(p.tolist(), d.tolist()))):
            els = np.nonzero((p == pe) & (d == de))[0]
            G = np.stack([edofs[e] for e in els])
            Eg = np.stack([E[off[e]:off[e + 1]] for e in els]).astype(np.longdouble)
            self.groups.append((pe, G, Eg, ks[(pe, de, nu)].astype(np.longdouble)))

    def apply(self, u):
        """K u for a full-length vector u (zeros at supported DOFs)."""
        u = np.asarray(u, dtype=np.longdouble)
        y = np.zeros(self.n_dof, dtype=np.longdouble)
        for pe, G, Eg, Ks in self.groups:
            ue = rigid_free(np.where(G >= 0, u[np.maximum(G, 0)], 0), pe)
            ye = np.einsum("ns,nsi->ni", Eg, np.einsum("sij,nj->nsi", Ks, ue))
            m = G >= 0
            np.add.at(y, G[m], ye[m])
        return y


def refined_solve(op, fi, lu, b, max_rounds=30):
    """Factor solve plus iterative refinement with a longdouble residual
    b - (K u)[fi] from the element operator; stops when the correction is
    below 1e-15 of u."""
    bl = b.astype(np.longdouble)
    u = np.zeros(op.n_dof, dtype=np.longdouble)
    u[fi] = lu.solve(b)
    for _ in range(max_rounds):
        r = bl - op.apply(u)[fi]
        du = lu.solve(np.asarray(r, dtype=np.float64))
        u[fi] += du.astype(np.longdouble)
        nu = float(np.sqrt(np.sum(u * u)))
        if nu == 0.0 or float(np.linalg.norm(du)) <= 1e-15 * nu:
            break
    return u[fi]


def spring_matrix(space, springs):
    """Ground springs (vx, vy, comp, k) as a diagonal matrix on the global
    DOFs: the force inverter's input and output springs of Sec. 4.1 add
    k u_i^2 / 2 to the strain energy, i.e. k to K_ii."""
    diag = np.zeros(space.n_dof)
    for vx, vy, comp, k in springs:
        diag[2 * (vy * (space.nelx + 1) + vx) + comp] += k
    return sp.diags(diag).tocsr()


def oracle_solve(nelx, nely, p, d, rho, supports, loads, n_load_cases=1,
                 E0=1.0, Emin=1e-9, nu=0.3, q=3.0, want_K=False, springs=(), tables=None):
    """Full reference step: returns dict with
    u [L, n_dof] (zero at supported DOFs), c [L], g [L, n_cells] (dc/drho),
    w [L, n_cells] (u_e^T K_s u_e), plus bookkeeping.  Ground springs
    (vx, vy, comp, k) are added to K; they do not depend on rho, so g keeps
    its form.  tables: optional dict (p, d, nu) -> K_s to use instead of
    computing them (for perturbation tests)."""
    K, space, edofs, off, ks = assemble(nelx, nely, p, d, rho, E0, Emin, q, nu,
                                        ks_cache=dict(tables) if tables else None)
    if len(springs):
        S = spring_matrix(space, springs)
        if np.any(S.diagonal()[~free_mask(space, supports)] != 0.0):
            raise ValueError("a spring acts on a supported DOF")
        K = (K + S).tocsr()
    free = free_mask(space, supports)
    f = load_vectors(space, loads, n_load_cases)
    if np.any(f[:, ~free] != 0.0):
        raise ValueError("a point load acts on a supported DOF")
    fi = np.nonzero(free)[0]
    Kff = K[fi][:, fi].tocsc()
    # K_ff is symmetric positive definite: symmetric ordering, no pivoting.
    lu = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    L = n_load_cases
    u = np.zeros((L, space.n_dof))
    c = np.zeros(L)
    E_all = simp_modulus(np.asarray(rho, dtype=np.float64).ravel(), E0, Emin, q)
    op = ElementOperator(p, d, E_all, edofs, off, ks, nu, space.n_dof)
    if len(springs):  # the springs' diagonal joins the element operator
        sdiag = spring_matrix(space, springs).diagonal().astype(np.longdouble)
        base = op.apply
        op.apply = lambda v, base=base, sdiag=sdiag: base(v) + sdiag * np.asarray(v, dtype=np.longdouble)
    for lc in range(L):
        ul = refined_solve(op, fi, lu, f[lc, fi])
        u[lc, fi] = np.asarray(ul, dtype=np.float64)
        c[lc] = float(np.dot(f[lc, fi].astype(np.longdouble), ul))
    # sensitivities: g_{e,s} = -E'(rho_{e,s}) u_e^T K_s u_e
    p_arr = np.asarray(p, dtype=np.int64).ravel()
    d_arr = np.asarray(d, dtype=np.int64).ravel()
    rho = np.asarray(rho, dtype=np.float64).ravel()
    dE = simp_modulus_derivative(rho, E0, Emin, q)
    w = np.zeros((L, rho.size))
    for e in range(nelx * nely):
        Ks = ks[(int(p_arr[e]), int(d_arr[e]), nu)]
        G = edofs[e]
        for lc in range(L):
            ue = rigid_free(np.where(G >= 0, u[lc, np.maximum(G, 0)], 0.0), int(p_arr[e]))
            w[lc, off[e]:off[e + 1]] = np.einsum("i,sij,j->s", ue, Ks, ue)
    g = -dE[None, :] * w
    out = dict(u=u, c=c, g=g, w=w, n_dof=space.n_dof, n_free=int(free.sum()), free=free,
               space=space, f=f)
    if want_K:
        out["K"] = K
    return out
