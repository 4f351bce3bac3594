"""Exact rational stiffness of the hierarchic Q_p element, for pinning the
oracle.  Independent route: polynomials with Fraction coefficients, Legendre
polynomials from Bonnet's recurrence, integrals by exact antiderivatives (no
quadrature), separable 2D integrals over each density cell.

Element: unit square, reference xi = 2x - 1 (d/dx = 2 d/dxi, dx = dxi / 2).
1D functions: (1 - xi)/2, (1 + xi)/2, and int_{-1}^{xi} P_{k-1} for k >= 2.
"""

from fractions import Fraction as F


def padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]


def pscale(a, s):
    return [s * c for c in a]


def pmul(a, b):
    out = [F(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def pder(a):
    return [i * a[i] for i in range(1, len(a))] or [F(0)]


def pint(a):
    """Antiderivative with zero constant term."""
    return [F(0)] + [a[i] / (i + 1) for i in range(len(a))]


def peval(a, x):
    v = F(0)
    for c in reversed(a):
        v = v * x + c
    return v


def legendre(n):
    """P_0..P_n by Bonnet: (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    P = [[F(1)], [F(0), F(1)]]
    for k in range(1, n):
        P.append(padd(pscale(pmul([F(0), F(1)], P[k]), F(2 * k + 1, k + 1)), pscale(P[k - 1], F(-k, k + 1))))
    return P[: n + 1]


def basis(p):
    """Hierarchic 1D basis in xi, as coefficient lists."""
    P = legendre(max(p, 1))
    out = [[F(1, 2), F(-1, 2)], [F(1, 2), F(1, 2)]]
    for k in range(2, p + 1):
        A = pint(P[k - 1])
        A = padd(A, [-peval(A, F(-1))])  # zero at xi = -1
        out.append(A)
    return out


def integral(a, lo, hi):
    A = pint(a)
    return peval(A, hi) - peval(A, lo)


def subcell_stiffness_exact(p, d, nu=F(3, 10)):
    """[S][ne][ne] Fractions: K_s = int_cell B^T D0 B over cell s = sy*d + sx."""
    n1 = p + 1
    ne = 2 * n1 * n1
    c = 1 / (1 - nu * nu)
    D = [[c, c * nu, 0], [c * nu, c, 0], [0, 0, c * (1 - nu) / 2]]
    phi = basis(p)
    dphi = [pder(f) for f in phi]
    out = []
    for sy in range(d):
        for sx in range(d):
            xlo, xhi = F(-1) + F(2 * sx, d), F(-1) + F(2 * (sx + 1), d)
            ylo, yhi = F(-1) + F(2 * sy, d), F(-1) + F(2 * (sy + 1), d)
            # 1D integrals in reference coordinates; each carries dx = dxi/2
            def I(f, g, lo, hi):
                return integral(pmul(f, g), lo, hi) / 2
            vv_x = [[I(phi[i], phi[k], xlo, xhi) for k in range(n1)] for i in range(n1)]
            dv_x = [[I(dphi[i], phi[k], xlo, xhi) * 2 for k in range(n1)] for i in range(n1)]  # d/dx = 2 d/dxi
            dd_x = [[I(dphi[i], dphi[k], xlo, xhi) * 4 for k in range(n1)] for i in range(n1)]
            vv_y = [[I(phi[i], phi[k], ylo, yhi) for k in range(n1)] for i in range(n1)]
            dv_y = [[I(dphi[i], phi[k], ylo, yhi) * 2 for k in range(n1)] for i in range(n1)]
            dd_y = [[I(dphi[i], dphi[k], ylo, yhi) * 4 for k in range(n1)] for i in range(n1)]
            K = [[F(0)] * ne for _ in range(ne)]
            for ja in range(n1):
                for ia in range(n1):
                    a = ja * n1 + ia
                    for jb in range(n1):
                        for ib in range(n1):
                            b = jb * n1 + ib
                            # integrals of products of derivatives of N_a = phi_ia(x) phi_ja(y)
                            xx = dd_x[ia][ib] * vv_y[ja][jb]      # Nx_a Nx_b
                            yy = vv_x[ia][ib] * dd_y[ja][jb]      # Ny_a Ny_b
                            xy = dv_x[ia][ib] * dv_y[jb][ja]      # Nx_a Ny_b
                            yx = dv_x[ib][ia] * dv_y[ja][jb]      # Ny_a Nx_b
                            # B columns: ux -> (Nx, 0, Ny), uy -> (0, Ny, Nx)
                            K[2 * a][2 * b] += D[0][0] * xx + D[2][2] * yy
                            K[2 * a][2 * b + 1] += D[0][1] * xy + D[2][2] * yx
                            K[2 * a + 1][2 * b] += D[1][0] * yx + D[2][2] * xy
                            K[2 * a + 1][2 * b + 1] += D[1][1] * yy + D[2][2] * xx
            out.append(K)
    return out


def mass_1d_exact(p):
    """m[i][k] = integral over the unit interval of phi_i phi_k (dx = dxi / 2)."""
    phi = basis(p)
    return [[integral(pmul(phi[i], phi[k]), F(-1), F(1)) / 2 for k in range(p + 1)] for i in range(p + 1)]


def moments_exact(beta, p):
    """Integrals over the unit element of the vector field b against every
    order-p function: b_c(xi, eta) = sum beta[c][i][j] xi^i eta^j (reference
    coordinates), result indexed 2a + c with a = j (p+1) + i of N_a =
    phi_i(xi) phi_j(eta)."""
    phi = basis(p)
    n1 = p + 1
    deg = len(beta[0])
    # 1D integrals of xi^m phi_i over [-1, 1], times 1/2 for dx = dxi / 2
    mono = [[integral(pmul([F(0)] * m + [F(1)], phi[i]), F(-1), F(1)) / 2 for i in range(n1)] for m in range(deg)]
    out = [F(0)] * (2 * n1 * n1)
    for c in range(2):
        for ja in range(n1):
            for ia in range(n1):
                acc = F(0)
                for mi in range(deg):
                    for mj in range(deg):
                        if beta[c][mi][mj]:
                            acc += beta[c][mi][mj] * mono[mi][ia] * mono[mj][ja]
                out[2 * (ja * n1 + ia) + c] = acc
    return out


def solve_exact(A, b):
    """Gauss-Jordan elimination with Fractions (A nonsingular)."""
    n = len(b)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [vr - fac * vc for vr, vc in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def pinned_solve_exact(K, f, pinned, values):
    """u with u[pinned] = values and (K u)[free] = f[free]."""
    n = len(f)
    free = [i for i in range(n) if i not in pinned]
    u = [F(0)] * n
    for k, v in zip(pinned, values):
        u[k] = v
    rhs = [f[i] - sum(K[i][k] * u[k] for k in pinned) for i in free]
    sol = solve_exact([[K[i][j] for j in free] for i in free], rhs)
    for i, v in zip(free, sol):
        u[i] = v
    return u
