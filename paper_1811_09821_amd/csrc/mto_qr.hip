// QR-error indicator of Sec. 3.2.3 (Eq. (9)): per element, the strain
// energy of the order-(p+1) element problem under the element's own load,
// against the order-p energy.
//
// One workgroup per element (all load cases of its instance share one
// factorisation):
//   1. K' = sum_s E_s K_s^(p+1) in LDS as a packed lower triangle, from the
//      order-(p+1) cell tables (packed the same way);
//   2. per load case, u_e from the free-DOF vector, minus the rigid motion
//      that the three pinned DOFs carry (vertex (0,0) x and y, vertex (1,0)
//      y), so that the pinned values are zero; f = K^(p) u_e, read from the
//      embedded block of K' (the hierarchic order-p functions are order-(p+1)
//      functions, and both matrices are integrated exactly, so that block is
//      K^(p)); J^(p) = u_e . f / 2;
//   3. the pinned rows and columns of K' are replaced by identity rows and
//      K' is factored in place (right-looking Cholesky, two barriers per
//      column);
//   4. one wave per load case solves K' u' = f' (f on the embedded DOFs; on
//      the new ones the integrals of the order-p load field against the new
//      functions, by the tensor product of the 1D transfer t; zero on the
//      pinned ones) with the rows held in lanes,
//      then refines u' twice against a double-double residual computed from
//      an unfactored copy of K', J^(p+1) = f' . u' / 2 (the load is
//      self-equilibrated, so the pinned DOFs carry no reaction and the rigid
//      motion removed in 2 changes neither energy), eps = 1 - J^(p) / J^(p+1),
//      or 0 if J^(p+1) = 0.
// eps is a small difference of two energies wherever the order-p field is
// already good, and the cell moduli inside one element can differ by 1e9, so
// f, both energies and the residuals are accumulated in double-double.

#include <hip/hip_runtime.h>

#include "mto_internal.hpp"
#include "mto_kernels.hpp"

namespace mto {
namespace {

constexpr int QR_BLOCK = 256;
constexpr int QR_LOADS = 8;  // load cases per pass over one factorisation

__device__ __forceinline__ int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// order-(p+1) local DOF of order-p local DOF 2 (j (p+1) + i) + c
template <int P>
__device__ __forceinline__ int emb(int d) {
  const int a = d >> 1, i = a % (P + 1), j = a / (P + 1);
  return 2 * (j * (P + 2) + i) + (d & 1);
}

// the order-p local DOF carried by order-(p+1) DOF r, or -1 for a new function
template <int P>
__device__ __forceinline__ int unemb(int r) {
  const int a = r >> 1, i = a % (P + 2), j = a / (P + 2);
  return (i <= P && j <= P) ? 2 * (j * (P + 1) + i) + (r & 1) : -1;
}

__device__ __forceinline__ bool pinned(int r) { return r == 0 || r == 1 || r == 3; }

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

#pragma clang fp contract(off)
// (hi, lo) += a * b, error-free product and two-sum
__device__ __forceinline__ void dd_fma(double a, double b, double& hi, double& lo) {
  const double p = a * b;
  const double e = fma(a, b, -p);
  const double s = hi + p;
  const double bb = s - hi;
  const double t = (hi - (s - bb)) + (p - bb);
  hi = s;
  lo += t + e;
}
// (hi, lo) += v
__device__ __forceinline__ void dd_add(double v, double& hi, double& lo) {
  const double s = hi + v;
  const double bb = s - hi;
  lo += (hi - (s - bb)) + (v - bb);
  hi = s;
}
// sum over the wave of (hi, lo) pairs, rounded
__device__ __forceinline__ double wave_sum_dd(double hi, double lo) {
  for (int o = 32; o > 0; o >>= 1) {
    const double h2 = __shfl_xor(hi, o), l2 = __shfl_xor(lo, o);
    dd_add(h2, hi, lo);
    lo += l2;
  }
  return hi + lo;
}
#pragma clang fp contract(on)

template <int P>
__global__ __launch_bounds__(QR_BLOCK) void k_qr(QrGroupDev g, const double* __restrict__ E,
                                                 const double* __restrict__ x, const SysDesc* __restrict__ sys,
                                                 const int32_t* __restrict__ inst_sys0,
                                                 const int32_t* __restrict__ inst_L,
                                                 const int64_t* __restrict__ inst_eoff,
                                                 const int32_t* __restrict__ inst_nel, double* __restrict__ eps) {
  constexpr int N1 = P + 1, NE = 2 * N1 * N1, NQ = 2 * (P + 2) * (P + 2), NT = NQ * (NQ + 1) / 2;
  static_assert(NQ <= 128, "rows are held two per lane");
  __shared__ double Kq[NT];   // K', then its Cholesky factor
  __shared__ double Kc[NT];   // K' with the identity rows, for the residuals
  __shared__ double Dinv[NQ];
  __shared__ double Es[MTO_MAX_D * MTO_MAX_D];
  __shared__ double U[QR_LOADS][NE];
  __shared__ double UD[QR_LOADS][NE];
  __shared__ double F[QR_LOADS][NE];   // f = K^(p) u, high and low parts
  __shared__ double Fl[QR_LOADS][NE];
  __shared__ double Xs[QR_BLOCK / 64][NQ];
  __shared__ double Jp[QR_LOADS];
  const int k = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int inst = g.einst[k], e = g.eid[k];
  const int64_t c0 = g.cell[k];
  const int nL = inst_L[inst], s0 = inst_sys0[inst], nel = inst_nel[inst];
  if (tid < g.S) Es[tid] = E[c0 + tid];
  __syncthreads();
  for (int l0 = 0; l0 < nL; l0 += QR_LOADS) {  // uniform
    const int nl = min(QR_LOADS, nL - l0);
    for (int idx = tid; idx < NT; idx += QR_BLOCK) {
      double acc = 0.0;
      for (int s = 0; s < g.S; ++s) acc = fma(Es[s], g.tab[(size_t)s * NT + idx], acc);
      Kq[idx] = acc;
    }
    for (int idx = tid; idx < nl * NE; idx += QR_BLOCK) {
      const int l = idx / NE, j = idx - l * NE;
      const int gi = g.gidx[(size_t)j * g.npad + k];
      U[l][j] = gi >= 0 ? x[sys[s0 + l0 + l].dof_off + gi] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < nl * NE; idx += QR_BLOCK) {
      const int l = idx / NE, j = idx - l * NE;
      // rigid motion (a - th y, b + th x) through the pinned values: a = u_x(0,0), b = u_y(0,0), th = u_y(1,0) - b
      const double a = U[l][0], b = U[l][1], th = U[l][3] - U[l][1];
      const int as = j >> 1, i1 = as % N1, j1 = as / N1;
      double v = U[l][j];
      if (i1 <= 1 && j1 <= 1) v -= (j & 1) ? b + th * i1 : a - th * j1;
      UD[l][j] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < nl * NE; idx += QR_BLOCK) {
      const int l = idx / NE, i = idx - l * NE;
      const int ei = emb<P>(i);
      double hi = 0.0, lo = 0.0;
      for (int j = 0; j < NE; ++j) dd_fma(Kq[tri(ei, emb<P>(j))], UD[l][j], hi, lo);
      const double sh = hi + lo;
      F[l][i] = sh;
      Fl[l][i] = lo - (sh - hi);
    }
    __syncthreads();
    for (int l = wave; l < nl; l += QR_BLOCK / 64) {
      double hi = 0.0, lo = 0.0;
      for (int i = lane; i < NE; i += 64) {
        dd_fma(UD[l][i], F[l][i], hi, lo);
        dd_fma(UD[l][i], Fl[l][i], hi, lo);
      }
      const double v = wave_sum_dd(hi, lo);
      if (lane == 0) Jp[l] = 0.5 * v;
    }
    for (int i = tid; i < NQ; i += QR_BLOCK) {  // identity rows and columns at the pinned DOFs
      const int pins[3] = {0, 1, 3};
      for (int c : pins) Kq[tri(i, c)] = i == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < NT; idx += QR_BLOCK) Kc[idx] = Kq[idx];
    __syncthreads();
    for (int kk = 0; kk < NQ; ++kk) {
      const double dkk = sqrt(Kq[tri(kk, kk)]);
      const double rinv = 1.0 / dkk;
      for (int i = kk + 1 + tid; i < NQ; i += QR_BLOCK) Kq[tri(i, kk)] *= rinv;
      __syncthreads();
      if (tid == 0) {
        Kq[tri(kk, kk)] = dkk;
        Dinv[kk] = rinv;
      }
      const int m = NQ - 1 - kk, cnt = m * (m + 1) / 2;
      for (int idx = tid; idx < cnt; idx += QR_BLOCK) {
        int ii = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
        while ((ii + 1) * (ii + 2) / 2 <= idx) ++ii;
        while (ii * (ii + 1) / 2 > idx) --ii;
        const int r = kk + 1 + ii, c = kk + 1 + (idx - ii * (ii + 1) / 2);
        Kq[tri(r, c)] = fma(-Kq[r * (r + 1) / 2 + kk], Kq[c * (c + 1) / 2 + kk], Kq[tri(r, c)]);
      }
      __syncthreads();
    }
    for (int l = wave; l < nl; l += QR_BLOCK / 64) {
      // rows lane and lane + 64
      double rh[2], rl[2], b[2], xv[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = lane + 64 * h, o = r < NQ ? unemb<P>(r) : -1;
        const bool on = o >= 0 && !pinned(r);
        rh[h] = on ? F[l][o] : 0.0;
        rl[h] = on ? Fl[l][o] : 0.0;
        if (r < NQ && o < 0) {  // a new function: phi_i(x) phi_j(y) with i or j = P + 1
          const int a = r >> 1, c = r & 1, i = a % (P + 2), j = a / (P + 2);
          double hi = 0.0, lo = 0.0;
          if (i == P + 1 && j == P + 1) {
            for (int jj = 0; jj <= P; ++jj) {
              double gh = 0.0, gl = 0.0;
              for (int ii = 0; ii <= P; ++ii) {
                const int q = 2 * (jj * (P + 1) + ii) + c;
                dd_fma(g.t[ii], F[l][q], gh, gl);
                gl = fma(g.t[ii], Fl[l][q], gl);
              }
              dd_fma(g.t[jj], gh, hi, lo);
              lo = fma(g.t[jj], gl, lo);
            }
          } else {
            const bool alongx = i == P + 1;  // the transfer acts in x (j <= P) or in y (i <= P)
            for (int k = 0; k <= P; ++k) {
              const int q = alongx ? 2 * (j * (P + 1) + k) + c : 2 * (k * (P + 1) + i) + c;
              dd_fma(g.t[k], F[l][q], hi, lo);
              lo = fma(g.t[k], Fl[l][q], lo);
            }
          }
          const double sh = hi + lo;
          rh[h] = sh;
          rl[h] = lo - (sh - hi);
        }
        b[h] = rh[h];
        xv[h] = 0.0;
      }
      for (int round = 0; round < 3; ++round) {  // a solve and two refinements
        if (round > 0) {  // b = f' - K' x in double-double, rounded
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (lane + 64 * h < NQ) Xs[wave][lane + 64 * h] = xv[h];
          __builtin_amdgcn_s_waitcnt(0xC07F);
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = lane + 64 * h;
            double hi = rh[h], lo = rl[h];
            if (r < NQ)
              for (int j = 0; j < NQ; ++j) dd_fma(-Kc[tri(r, j)], Xs[wave][j], hi, lo);
            b[h] = hi + lo;
          }
          __builtin_amdgcn_s_waitcnt(0xC07F);
          __builtin_amdgcn_wave_barrier();
        }
        for (int kk = 0; kk < NQ; ++kk) {  // forward: L y = b
          const double y = readlane_d((kk >> 6 ? b[1] : b[0]) * Dinv[kk], kk & 63);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = lane + 64 * h;
            if (r == kk) b[h] = y;
            else if (r > kk && r < NQ) b[h] = fma(-Kq[r * (r + 1) / 2 + kk], y, b[h]);
          }
        }
        for (int kk = NQ - 1; kk >= 0; --kk) {  // backward: L^T d = y
          const double xk = readlane_d((kk >> 6 ? b[1] : b[0]) * Dinv[kk], kk & 63);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = lane + 64 * h;
            if (r == kk) b[h] = xk;
            else if (r < kk) b[h] = fma(-Kq[kk * (kk + 1) / 2 + r], xk, b[h]);
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) xv[h] += b[h];
      }
      double jh = 0.0, jl = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        dd_fma(rh[h], xv[h], jh, jl);
        dd_fma(rl[h], xv[h], jh, jl);
      }
      const double Jq = 0.5 * wave_sum_dd(jh, jl);
      if (lane == 0) {
        const int L = l0 + l;
        eps[inst_eoff[inst] + (int64_t)L * nel + e] = Jq > 0.0 ? 1.0 - Jp[l] / Jq : 0.0;
      }
    }
    __syncthreads();  // the next pass rebuilds K'
  }
}

}  // namespace

void launch_qr(const QrGroupDev& g, const double* E, const double* x, const SysDesc* sys, const int32_t* inst_sys0,
               const int32_t* inst_L, const int64_t* inst_eoff, const int32_t* inst_nel, double* eps,
               hipStream_t st) {
  if (g.n_elems == 0) return;
  const dim3 grid(g.n_elems), block(QR_BLOCK);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_qr<1>, grid, block, 0, st, g, E, x, sys, inst_sys0, inst_L, inst_eoff, inst_nel, eps); break;
    case 2: hipLaunchKernelGGL(k_qr<2>, grid, block, 0, st, g, E, x, sys, inst_sys0, inst_L, inst_eoff, inst_nel, eps); break;
    case 3: hipLaunchKernelGGL(k_qr<3>, grid, block, 0, st, g, E, x, sys, inst_sys0, inst_L, inst_eoff, inst_nel, eps); break;
    default: hipLaunchKernelGGL(k_qr<4>, grid, block, 0, st, g, E, x, sys, inst_sys0, inst_L, inst_eoff, inst_nel, eps); break;
  }
}

}  // namespace mto
