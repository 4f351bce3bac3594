// Refinement indicators of Sec. 3.2 and the dp update of Sec. 3.3.
//
// Analysis indicator (Sec. 3.2.1, Kelly): Gamma^a of an element is the sum
// over its interior edges F of c_F * integral_F |[du/dn]|^2 ds, c_F =
// h_F / (2 p_F), h_F the element diagonal (sqrt 2 in element units), p_F the
// larger order of the two elements; the integral is exact Gauss-Legendre with
// p_F + 1 points (the squared jump has degree 2 p_F along the edge).  One
// thread per (element, system); each thread gathers its own and its
// neighbours' element vectors, so an edge is integrated once from each side
// and no atomics or edge arrays are needed.
//
// Density indicator (Sec. 3.2.2): one thread per element sums the four
// cases over its cells.
//
// dp update (Sec. 3.3, steps 2-4): host code (ranking, flags, smoothing).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "mto_internal.hpp"
#include "mto_kernels.hpp"

namespace mto {
namespace {

constexpr int AD_BLOCK = 64;

// Gauss-Legendre rules with n = 2..5 points on [-1, 1] (nodes and weights of
// the n-point rule: roots of P_n, weights 2 / ((1 - t^2) P_n'(t)^2))
__device__ __forceinline__ void gauss_rule(int n, int q, double& t, double& w) {
  switch (n) {
    case 2:
      t = q == 0 ? -0.57735026918962576451 : 0.57735026918962576451;
      w = 1.0;
      break;
    case 3: {
      const double tt[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
      const double ww[3] = {0.55555555555555555556, 0.88888888888888888889, 0.55555555555555555556};
      t = tt[q];
      w = ww[q];
      break;
    }
    case 4: {
      const double tt[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                            0.86113631159405257522};
      const double ww[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                            0.34785484513745385737};
      t = tt[q];
      w = ww[q];
      break;
    }
    default: {
      const double tt[5] = {-0.90617984593866399280, -0.53846931010568309104, 0.0, 0.53846931010568309104,
                            0.90617984593866399280};
      const double ww[5] = {0.23692688505618908751, 0.47862867049936646804, 0.56888888888888888889,
                            0.47862867049936646804, 0.23692688505618908751};
      t = tt[q];
      w = ww[q];
      break;
    }
  }
}

// hierarchic 1D functions of order p at t: phi[k] and phi'[k], k = 0..p
__device__ __forceinline__ void basis(int p, double t, double* f, double* df) {
  double P0 = 1.0, P1 = t;  // Legendre P_{k-2}, P_{k-1}
  f[0] = 0.5 * (1.0 - t);
  df[0] = -0.5;
  f[1] = 0.5 * (1.0 + t);
  df[1] = 0.5;
  for (int k = 2; k <= p; ++k) {
    const double Pk = ((2 * k - 1) * t * P1 - (k - 1) * P0) / k;
    f[k] = (Pk - P0) / (2 * k - 1);
    df[k] = P1;
    P0 = P1;
    P1 = Pk;
  }
}

// outward normal derivative (both components) of the element field ue of
// order p on side s (0 left, 1 right, 2 bottom, 3 top) at tangential t
__device__ void grad_normal(const double* ue, int p, int s, double t, double& gx, double& gy) {
  double ft[MTO_MAX_P + 1], dft[MTO_MAX_P + 1], ff[MTO_MAX_P + 1], dff[MTO_MAX_P + 1];
  basis(p, t, ft, dft);
  basis(p, (s == 0 || s == 2) ? -1.0 : 1.0, ff, dff);
  const double sign = (s == 1 || s == 3) ? 2.0 : -2.0;  // d/dx = 2 d/dxi, outward sign
  gx = gy = 0.0;
  const int n1 = p + 1;
  for (int j = 0; j < n1; ++j)
    for (int i = 0; i < n1; ++i) {
      const double v = (s <= 1) ? dff[i] * ft[j] : ft[i] * dff[j];
      const int a = j * n1 + i;
      gx = fma(ue[2 * a], v, gx);
      gy = fma(ue[2 * a + 1], v, gy);
    }
  gx *= sign;
  gy *= sign;
}

__device__ void gather_elem(const AdaptDev& a, int64_t gel, const double* __restrict__ xs, double* ue, int& p) {
  const int g = a.el_group[gel], k = a.el_col[gel];
  const GroupDev& G = a.groups[g];
  p = G.p;
  const int ne = 2 * (p + 1) * (p + 1);
  for (int j = 0; j < ne; ++j) {
    const int gi = G.gidx[(size_t)j * G.npad + k];
    ue[j] = gi >= 0 ? xs[gi] : 0.0;
  }
}

__global__ __launch_bounds__(AD_BLOCK) void k_kelly(AdaptDev a, const SysDesc* __restrict__ sys,
                                                    const double* __restrict__ x, double* __restrict__ gamma) {
  const int sidx = blockIdx.y;
  const SysDesc& sd = sys[sidx];
  const int inst = sd.inst, nelx = a.nelx[inst], nely = a.nely[inst], nel = nelx * nely;
  const int e = blockIdx.x * AD_BLOCK + threadIdx.x;
  if (e >= nel) return;
  const double* __restrict__ xs = x + sd.dof_off;
  const int64_t base = a.el_base[inst];
  constexpr int NEMAX = 2 * (MTO_MAX_P + 1) * (MTO_MAX_P + 1);
  double ue[NEMAX], uf[NEMAX];
  int pe, pf;
  gather_elem(a, base + e, xs, ue, pe);
  const int ex = e % nelx, ey = e / nelx;
  double total = 0.0;
  for (int s = 0; s < 4; ++s) {
    const int fx = ex + (s == 0 ? -1 : s == 1 ? 1 : 0), fy = ey + (s == 2 ? -1 : s == 3 ? 1 : 0);
    if (fx < 0 || fx >= nelx || fy < 0 || fy >= nely) continue;  // boundary edge: no jump
    gather_elem(a, base + fy * nelx + fx, xs, uf, pf);
    const int pF = max(pe, pf), so = s ^ 1;  // the neighbour's side facing this edge
    double integral = 0.0;
    for (int q = 0; q <= pF; ++q) {
      double t, w, ax, ay, bx, by;
      gauss_rule(pF + 1, q, t, w);
      grad_normal(ue, pe, s, t, ax, ay);
      grad_normal(uf, pf, so, t, bx, by);
      const double jx = ax + bx, jy = ay + by;  // outward normals are opposite
      integral = fma(0.5 * w, jx * jx + jy * jy, integral);  // ds = dt / 2
    }
    total = fma(1.4142135623730950488 / (2.0 * pF), integral, total);
  }
  gamma[a.inst_eoff[inst] + (int64_t)sd.load * nel + e] = total;
}

__global__ __launch_bounds__(AD_BLOCK) void k_density_ind(AdaptDev a, const double* __restrict__ rho,
                                                          DensityBounds b, double* __restrict__ gamma,
                                                          int64_t n_el) {
  const int64_t gel = (int64_t)blockIdx.x * AD_BLOCK + threadIdx.x;
  if (gel >= n_el) return;
  const int g = a.el_group[gel], k = a.el_col[gel];
  const GroupDev& G = a.groups[g];
  const int n = G.S;
  const double* __restrict__ r = rho + G.cell[k];
  double acc = 0.0;
  for (int j = 0; j < n; ++j) {
    const double v = r[j];
    if (b.rl <= v && v <= b.avg) acc += (v - b.rl) / n;
    if (b.avg < v && v <= b.ru) acc += (b.ru - v) / n;
    if (v <= b.cl) acc -= (b.cl - v) / n;
    if (v >= b.cu) acc -= (v - b.cu) / n;
  }
  gamma[gel] = acc;
}

}  // namespace

void launch_kelly(const AdaptDev& a, const SysDesc* sys, int n_sys, int nel_max, const double* x, double* gamma,
                  hipStream_t st) {
  if (n_sys == 0 || nel_max == 0) return;
  hipLaunchKernelGGL(k_kelly, dim3((nel_max + AD_BLOCK - 1) / AD_BLOCK, n_sys), dim3(AD_BLOCK), 0, st, a, sys, x,
                     gamma);
}

void launch_density_indicator(const AdaptDev& a, const double* rho, const DensityBounds& b, double* gamma,
                              int64_t n_el, hipStream_t st) {
  if (n_el == 0) return;
  hipLaunchKernelGGL(k_density_ind, dim3((unsigned)((n_el + AD_BLOCK - 1) / AD_BLOCK)), dim3(AD_BLOCK), 0, st, a,
                     rho, b, gamma, n_el);
}

}  // namespace mto

// ---- host: dp update (Sec. 3.3) ----

namespace {

// elements in ascending order of v, ties by element index
std::vector<int> ranking(const double* v, int n) {
  std::vector<int> o(n);
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return v[a] < v[b]; });
  return o;
}

// Raise the lower order of neighbours until they differ by at most 2:
// (p_max - p_min - 2) passes, rows bottom to top, each element against its
// right and upper neighbour, in place (Sec. 3.3, step 3c).
void smooth(std::vector<int>& p, int nelx, int nely) {
  const auto mm = std::minmax_element(p.begin(), p.end());
  const int passes = std::max(0, *mm.second - *mm.first - 2);
  for (int it = 0; it < passes; ++it)
    for (int ey = 0; ey < nely; ++ey)
      for (int ex = 0; ex < nelx; ++ex) {
        const int e = ey * nelx + ex;
        const int nb[2] = {ex + 1 < nelx ? e + 1 : -1, ey + 1 < nely ? e + nelx : -1};
        for (int f : nb) {
          if (f < 0) continue;
          if (p[e] < p[f] - 2) p[e] = p[f] - 2;
          else if (p[f] < p[e] - 2) p[f] = p[e] - 2;
        }
      }
}

}  // namespace

extern "C" {

int mto_dp_update(int32_t nelx, int32_t nely, const int8_t* p_in, const double* gamma_a, const double* gamma_d,
                  const mto_dp_params* prm, int8_t* p_out, int8_t* theta_out, int32_t* design_points,
                  int32_t* cells_per_element) {
  mto::clear_error();
  if (nelx < 1 || nely < 1 || !p_in || !gamma_a || !gamma_d || !prm || !p_out || !theta_out || !design_points ||
      !cells_per_element)
    return mto::set_error(MTO_EINVAL, "dp update: bad arguments");
  if (prm->p_max < 1 || prm->p_max > 126 || prm->d_max < 1 || !(prm->frac_a_refine >= 0 && prm->frac_a_refine <= 1) ||
      !(prm->frac_a_coarsen >= 0 && prm->frac_a_coarsen <= 1) || !(prm->frac_d_refine >= 0 && prm->frac_d_refine <= 1) ||
      !(prm->frac_d_coarsen >= 0 && prm->frac_d_coarsen <= 1))
    return mto::set_error(MTO_EINVAL, "dp update: parameters out of range");
  const int n = nelx * nely;
  std::vector<int> p(n), th(n, 0);
  for (int k = 0; k < n; ++k) {
    if (p_in[k] < 1) return mto::set_error(MTO_EINVAL, "dp update: p < 1");
    p[k] = p_in[k];
  }
  // step 2: analysis indicator, bottom fraction coarsened, top fraction refined
  {
    const std::vector<int> o = ranking(gamma_a, n);
    const int nc = (int)std::floor(prm->frac_a_coarsen * n), nr = (int)std::floor(prm->frac_a_refine * n);
    for (int k = 0; k < nc; ++k) th[o[k]] = -1;
    for (int k = n - nr; k < n; ++k) th[o[k]] = 1;
    for (int k = 0; k < n; ++k) p[k] = std::min(std::max(p[k] + th[k], 1), (int)prm->p_max);
  }
  // step 3: density indicator among the elements with Gamma^d < 0 (coarsen) and > 0 (refine)
  {
    const std::vector<int> o = ranking(gamma_d, n);
    std::vector<int> neg, pos;
    for (int k : o) {
      if (gamma_d[k] < 0.0) neg.push_back(k);
      else if (gamma_d[k] > 0.0) pos.push_back(k);
    }
    const int nc = (int)std::floor(prm->frac_d_coarsen * neg.size());
    const int nr = (int)std::floor(prm->frac_d_refine * pos.size());
    for (int m = 0; m < nc; ++m) {
      const int k = neg[m];
      if (p[k] == 1) th[k] = -2;
      else if (th[k] == 0) p[k] -= 1;
    }
    for (int m = (int)pos.size() - nr; m < (int)pos.size(); ++m) {
      const int k = pos[m];
      if (th[k] == 0 || th[k] == -1) p[k] = std::min(p[k] + 1, (int)prm->p_max);
    }
  }
  smooth(p, nelx, nely);
  int dmax = 0;
  for (int k = 0; k < n; ++k) {
    p_out[k] = (int8_t)p[k];
    theta_out[k] = (int8_t)th[k];
    const int dof = 2 * (p[k] + 1) * (p[k] + 1) - 3;  // element DOFs minus the rigid modes
    design_points[k] = th[k] == -2 ? 1 : std::min(dof, (int)prm->d_max);
    dmax = std::max(dmax, design_points[k]);
  }
  int side = 1;
  while (side * side < dmax) ++side;
  *cells_per_element = side * side;
  return MTO_OK;
}

int mto_qr_update(int32_t nel, const int8_t* p_in, const double* eps, double alpha_qr, int32_t p_max, int8_t* p_out) {
  mto::clear_error();
  if (nel < 0 || !p_in || !eps || !p_out || p_max < 1 || p_max > 126)
    return mto::set_error(MTO_EINVAL, "QR update: bad arguments");
  for (int k = 0; k < nel; ++k) p_out[k] = (int8_t)std::min((int)p_in[k] + (eps[k] > alpha_qr ? 1 : 0), (int)p_max);
  return MTO_OK;
}

}  // extern "C"
