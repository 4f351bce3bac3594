// Subcell stiffness tables K_s (Appendix B, composite integration over the
// density cells of one element) and their MFMA fragment layout.
//
// Element: unit square, reference coordinates (xi, eta) in [-1, 1]^2 with
// d/dx = 2 d/dxi and dx dy = dxi deta / 4.  Basis per direction: (1 - xi)/2,
// (1 + xi)/2 and the integrated Legendre polynomials
// L_k(xi) = (P_k(xi) - P_{k-2}(xi)) / (2k - 1) (so L_k' = P_{k-1}), k = 2..p.
// Local DOF 2a + c with a = j (p+1) + i for the function phi_i(xi) phi_j(eta).
// Material: plane-stress D0 of Sec. 2.2 (E = 1), unit thickness.
// Each K_s = int_cell B^T D0 B, by a (p+1) x (p+1) Gauss-Legendre rule mapped to
// the cell: exact, since the integrand has degree <= 2p per direction.
// Accumulation in long double, rounded once to double.

#include <cmath>
#include <utility>
#include <vector>

#include "mto_internal.hpp"

namespace mto {
namespace {

using ld = long double;

// Legendre P_0..P_n and derivatives at x by the three-term recurrence.
void legendre(int n, ld x, ld* P, ld* dP) {
  P[0] = 1;
  dP[0] = 0;
  if (n >= 1) {
    P[1] = x;
    dP[1] = 1;
  }
  for (int k = 1; k < n; ++k) {
    P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
}

// n-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, ld* x, ld* w) {
  const ld pi = 3.141592653589793238462643383279502884L;
  ld P[16], dP[16];
  for (int i = 0; i < n; ++i) {
    ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, P, dP);
      ld dz = P[n] / dP[n];
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    legendre(n, z, P, dP);
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dP[n] * dP[n]);
  }
}

// Hierarchic 1D shape functions phi_0..phi_p and derivatives at xi.
void shape_1d(int p, ld xi, ld* phi, ld* dphi) {
  ld P[16], dP[16];
  legendre(p, xi, P, dP);
  phi[0] = (1 - xi) / 2;
  dphi[0] = -0.5L;
  phi[1] = (1 + xi) / 2;
  dphi[1] = 0.5L;
  for (int k = 2; k <= p; ++k) {
    phi[k] = (P[k] - P[k - 2]) / (2 * k - 1);
    dphi[k] = P[k - 1];
  }
}

}  // namespace

std::vector<double> subcell_tables(int p, int d, double nu) {
  const int n1 = p + 1, ne = ne_of(p), S = d * d;
  std::vector<ld> acc((size_t)S * ne * ne, 0);
  const ld c = 1.0L / (1.0L - (ld)nu * nu);
  const ld D[3][3] = {{c, c * nu, 0}, {c * nu, c, 0}, {0, 0, c * (1 - (ld)nu) / 2}};
  ld gx[16], gw[16];
  gauss_legendre(n1, gx, gw);
  const ld h = 2.0L / d;
  std::vector<ld> B(3 * (size_t)ne);
  std::vector<ld> DB(3 * (size_t)ne);
  for (int sy = 0; sy < d; ++sy)
    for (int sx = 0; sx < d; ++sx) {
      ld* K = &acc[(size_t)(sy * d + sx) * ne * ne];
      for (int qy = 0; qy < n1; ++qy)
        for (int qx = 0; qx < n1; ++qx) {
          const ld xi = -1 + h * sx + h * (gx[qx] + 1) / 2;
          const ld eta = -1 + h * sy + h * (gx[qy] + 1) / 2;
          const ld wt = (h / 2) * gw[qx] * (h / 2) * gw[qy] / 4;  // includes dx dy = dxi deta / 4
          ld fx[16], dfx[16], fy[16], dfy[16];
          shape_1d(p, xi, fx, dfx);
          shape_1d(p, eta, fy, dfy);
          std::fill(B.begin(), B.end(), 0);
          for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
              const int a = j * n1 + i;
              const ld Nx = 2 * dfx[i] * fy[j];
              const ld Ny = 2 * fx[i] * dfy[j];
              B[0 * ne + 2 * a] = Nx;
              B[1 * ne + 2 * a + 1] = Ny;
              B[2 * ne + 2 * a] = Ny;
              B[2 * ne + 2 * a + 1] = Nx;
            }
          for (int r = 0; r < 3; ++r)
            for (int k = 0; k < ne; ++k)
              DB[r * ne + k] = D[r][0] * B[0 * ne + k] + D[r][1] * B[1 * ne + k] + D[r][2] * B[2 * ne + k];
          for (int i = 0; i < ne; ++i)
            for (int j = 0; j < ne; ++j)
              K[i * ne + j] += wt * (B[0 * ne + i] * DB[0 * ne + j] + B[1 * ne + i] * DB[1 * ne + j] +
                                     B[2 * ne + i] * DB[2 * ne + j]);
        }
    }
  std::vector<double> out(acc.size());
  for (size_t k = 0; k < acc.size(); ++k) out[k] = (double)acc[k];
  // exact symmetry (the integrand is symmetric; rounding of the products is not)
  for (int s = 0; s < S; ++s)
    for (int i = 0; i < ne; ++i)
      for (int j = 0; j < i; ++j) out[(size_t)s * ne * ne + i * ne + j] = out[(size_t)s * ne * ne + j * ne + i];
  return out;
}

std::vector<double> qr_load_transfer(int p) {
  // 1D mass matrix of the order-(p+1) functions on the unit interval
  // (dx = dxi / 2), exact with p + 2 Gauss points (degree 2p + 2)
  const int n = p + 2;
  ld gx[16], gw[16];
  gauss_legendre(n, gx, gw);
  std::vector<ld> m((size_t)n * n, 0);
  for (int q = 0; q < n; ++q) {
    ld phi[16], dphi[16];
    shape_1d(p + 1, gx[q], phi, dphi);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) m[(size_t)i * n + k] += gw[q] * phi[i] * phi[k] / 2;
  }
  // t solves m_p t = m[0..p][p+1] (m_p: the leading (p+1) x (p+1) block, the
  // order-p mass matrix), by Gaussian elimination with partial pivoting
  const int k1 = p + 1;
  std::vector<ld> A((size_t)k1 * (k1 + 1));
  for (int i = 0; i < k1; ++i) {
    for (int k = 0; k < k1; ++k) A[(size_t)i * (k1 + 1) + k] = m[(size_t)i * n + k];
    A[(size_t)i * (k1 + 1) + k1] = m[(size_t)i * n + (p + 1)];
  }
  for (int c = 0; c < k1; ++c) {
    int piv = c;
    for (int r = c + 1; r < k1; ++r)
      if (std::fabs(A[(size_t)r * (k1 + 1) + c]) > std::fabs(A[(size_t)piv * (k1 + 1) + c])) piv = r;
    for (int k = 0; k <= k1; ++k) std::swap(A[(size_t)c * (k1 + 1) + k], A[(size_t)piv * (k1 + 1) + k]);
    for (int r = 0; r < k1; ++r) {
      if (r == c) continue;
      const ld fac = A[(size_t)r * (k1 + 1) + c] / A[(size_t)c * (k1 + 1) + c];
      for (int k = c; k <= k1; ++k) A[(size_t)r * (k1 + 1) + k] -= fac * A[(size_t)c * (k1 + 1) + k];
    }
  }
  std::vector<double> t(k1);
  for (int i = 0; i < k1; ++i) t[i] = (double)(A[(size_t)i * (k1 + 1) + k1] / A[(size_t)i * (k1 + 1) + i]);
  return t;
}

std::vector<double> mfma_fragments(const std::vector<double>& ks, int p, int d) {
  const int ne = ne_of(p), nep = nep_of(p), mb = mb_of(p), S = d * d;
  const int T = S * nep / 4;
  std::vector<double> fr((size_t)T * mb * 64, 0.0);
  for (int t = 0; t < T; ++t)
    for (int b = 0; b < mb; ++b)
      for (int l = 0; l < 64; ++l) {
        const int row = b * 16 + (l % 16);
        const int k = 4 * t + l / 16;
        const int s = k / nep, j = k % nep;
        double v = 0.0;
        if (row < ne && j < ne) v = ks[(size_t)s * ne * ne + row * ne + j];
        fr[((size_t)t * mb + b) * 64 + l] = v;
      }
  return fr;
}

std::vector<double> staged_fragments(const std::vector<double>& ks, int p, int d) {
  const int ne = ne_of(p), nj = nep_of(p) / 4, mbm = mbm_of(p), tr = tr_of(p), frj = frj_of(p), S = d * d;
  std::vector<double> fr((size_t)S * nj * frj, 0.0);
  for (int s = 0; s < S; ++s)
    for (int jj = 0; jj < nj; ++jj) {
      double* f = &fr[((size_t)s * nj + jj) * frj];
      for (int b = 0; b < mbm; ++b)
        for (int l = 0; l < 64; ++l) {
          const int row = b * 16 + (l % 16), j = 4 * jj + l / 16;
          f[b * 64 + l] = (row < ne && j < ne) ? ks[(size_t)s * ne * ne + row * ne + j] : 0.0;
        }
      for (int kq = 0; kq < 4; ++kq)
        for (int r = 0; r < tr; ++r) {
          const int row = 16 * mbm + r, j = 4 * jj + kq;
          f[mbm * 64 + kq * tr + r] = (row < ne && j < ne) ? ks[(size_t)s * ne * ne + row * ne + j] : 0.0;
        }
    }
  return fr;
}

std::vector<double> vertex_fragments(const std::vector<double>& ks, int p, int d) {
  const int ne = ne_of(p), mb = mb_of(p), S = d * d;
  std::vector<double> fr((size_t)S * 2 * mb * 64, 0.0);
  for (int s = 0; s < S; ++s)
    for (int jj = 0; jj < 2; ++jj)
      for (int b = 0; b < mb; ++b)
        for (int l = 0; l < 64; ++l) {
          const int row = b * 16 + (l % 16), v = 4 * jj + l / 16;
          const int col = v < 4 ? v : 2 * (p + 1) + (v - 4);
          fr[(((size_t)s * 2 + jj) * mb + b) * 64 + l] = row < ne ? ks[(size_t)s * ne * ne + row * ne + col] : 0.0;
        }
  return fr;
}

}  // namespace mto
