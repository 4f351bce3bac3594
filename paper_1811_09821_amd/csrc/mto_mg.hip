// Geometric multigrid preconditioner for the PCG of the FEA step.
//
// Level 0 is the mixed-order hierarchic space itself (matrix-free, MFMA
// contraction).  Because the basis is hierarchic, the bilinear (Q1) space of
// the vertex functions is a subspace of it: level 1 is the vertex grid, the
// transfer is injection of the vertex DOFs, and the Galerkin operator
// A1 = P^T A0 P is the vertex-vertex block of K, assembled per element from
// sum_s E_s K_s[vertex rows, vertex columns].  Levels 2.. coarsen the vertex
// grid by two per direction (an odd element count keeps its last node), with
// bilinear prolongation P and Galerkin operators A_{l+1} = P^T A_l P, all in
// structured 9-point stencil form (nine 2 x 2 blocks per node).  Supported
// DOFs and DOFs whose prolongated basis vanishes are masked out of P and get
// identity rows.  Smoother: l1-Jacobi (diagonal sum_j |A_ij|), which needs no
// eigenvalue estimate and keeps the V-cycle symmetric positive definite; one
// pre- and one post-sweep per level.  The coarsest grid (<= 256 DOFs) is
// solved with a dense inverse formed once per design.

#include <hip/hip_runtime.h>

#include "mto_kernels.hpp"

namespace mto {
namespace {

constexpr int MGB = MG_CHUNK;

// Bilinear parents of fine node f on a 1D grid of nf elements (the coarse
// grid has ceil(nf / 2) elements; coarse node c sits on fine node min(2c, nf)).
__device__ __forceinline__ void parents1d(int f, int nf, int& c0, double& w0, int& c1, double& w1) {
  const int nc = (nf + 1) / 2;
  if (f == nf) {
    c0 = nc;
    w0 = 1.0;
    c1 = -1;
    w1 = 0.0;
  } else if ((f & 1) == 0) {
    c0 = f / 2;
    w0 = 1.0;
    c1 = -1;
    w1 = 0.0;
  } else {
    c0 = (f - 1) / 2;
    c1 = (f + 1) / 2;
    w0 = 0.5;
    w1 = 0.5;
  }
}

// Weight of coarse node c in fine node f (0 if not a parent).
__device__ __forceinline__ double weight1d(int f, int nf, int c) {
  int c0, c1;
  double w0, w1;
  parents1d(f, nf, c0, w0, c1, w1);
  return c0 == c ? w0 : (c1 == c ? w1 : 0.0);
}

__device__ __forceinline__ int fine_of(int c, int nf) { return min(2 * c, nf); }

__device__ __forceinline__ bool sys_running(const PcgDev& s, int sys) { return s.status[sys] == SYS_RUNNING; }

}  // namespace

// Level-1 operator: vertex-vertex blocks of the element matrices.
__global__ __launch_bounds__(MGB) void k_mg_assemble1(const MgChunk* __restrict__ chunks, const MgElem* __restrict__ elems,
                                                      const double* __restrict__ kv, const double* __restrict__ E,
                                                      const int32_t* __restrict__ vfree, double* __restrict__ A,
                                                      double* __restrict__ mask) {
  const MgChunk ch = chunks[blockIdx.x];
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int nx = ch.nx, ny = ch.ny;
  const int ix = n % (nx + 1), iy = n / (nx + 1);
  double blk[9][4];
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) blk[k][c] = 0.0;
  for (int dj = 0; dj < 2; ++dj)
    for (int di = 0; di < 2; ++di) {
      const int ex = ix - 1 + di, ey = iy - 1 + dj;
      if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
      const int i0 = ix - ex, j0 = iy - ey, a0 = 2 * j0 + i0;
      const MgElem el = elems[ch.elem_off + (int64_t)ey * nx + ex];
      for (int a1 = 0; a1 < 4; ++a1) {
        const int i1 = a1 & 1, j1 = a1 >> 1;
        const int k = (j1 - j0 + 1) * 3 + (i1 - i0 + 1);
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
        for (int sc = 0; sc < el.S; ++sc) {
          const double Es = E[el.cell_off + sc];
          const double* t = kv + el.kv_off + ((sc * 4 + a0) * 4 + a1) * 4;
          b0 = fma(Es, t[0], b0);
          b1 = fma(Es, t[1], b1);
          b2 = fma(Es, t[2], b2);
          b3 = fma(Es, t[3], b3);
        }
        blk[k][0] += b0;
        blk[k][1] += b1;
        blk[k][2] += b2;
        blk[k][3] += b3;
      }
    }
  const int64_t node = ch.op + n;
  double m[2];
  for (int c = 0; c < 2; ++c) m[c] = vfree[node * 2 + c] >= 0 ? 1.0 : 0.0;
  for (int k = 0; k < 9; ++k) {
    const int dx = k % 3 - 1, dy = k / 3 - 1;
    const int jx = ix + dx, jy = iy + dy;
    double mj[2] = {0.0, 0.0};
    if (jx >= 0 && jx <= nx && jy >= 0 && jy <= ny) {
      const int64_t jn = ch.op + (int64_t)jy * (nx + 1) + jx;
      mj[0] = vfree[jn * 2] >= 0 ? 1.0 : 0.0;
      mj[1] = vfree[jn * 2 + 1] >= 0 ? 1.0 : 0.0;
    }
    for (int c = 0; c < 2; ++c)
      for (int cc = 0; cc < 2; ++cc) {
        double v = blk[k][c * 2 + cc] * m[c] * mj[cc];
        if (k == 4 && c == cc && m[c] == 0.0) v = 1.0;
        A[node * 36 + k * 4 + c * 2 + cc] = v;
      }
  }
  mask[node * 2] = m[0];
  mask[node * 2 + 1] = m[1];
}

// l1-Jacobi inverse diagonal of a level: 1 / sum_j |A_ij|.
__global__ __launch_bounds__(MGB) void k_mg_l1(const MgChunk* __restrict__ chunks, const double* __restrict__ A,
                                               double* __restrict__ dinv) {
  const MgChunk ch = chunks[blockIdx.x];
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int64_t node = ch.op + n;
  for (int c = 0; c < 2; ++c) {
    double sum = 0.0;
    for (int k = 0; k < 9; ++k) sum += fabs(A[node * 36 + k * 4 + c * 2]) + fabs(A[node * 36 + k * 4 + c * 2 + 1]);
    dinv[node * 2 + c] = sum > 0.0 ? 1.0 / sum : 0.0;
  }
}

// Galerkin coarse operator A_c = P~^T A_f P~ (P~ = bilinear prolongation with
// the masked fine DOFs zeroed), one coarse node per thread.
__global__ __launch_bounds__(MGB) void k_mg_rap(const MgChunk* __restrict__ chunks, double* __restrict__ A,
                                                double* __restrict__ mask) {
  const MgChunk ch = chunks[blockIdx.x];
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int nx = ch.nx, fnx = ch.fnx, fny = ch.fny;
  const int cx = n % (nx + 1), cy = n / (nx + 1);
  double acc[9][4];
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[k][c] = 0.0;
  const int fxc0 = fine_of(cx, fnx), fyc0 = fine_of(cy, fny);
  for (int oy = -1; oy <= 1; ++oy) {
    const int fy = fyc0 + oy;
    if (fy < 0 || fy > fny) continue;
    const double wy = weight1d(fy, fny, cy);
    if (wy == 0.0) continue;
    for (int ox = -1; ox <= 1; ++ox) {
      const int fx = fxc0 + ox;
      if (fx < 0 || fx > fnx) continue;
      const double wx = weight1d(fx, fnx, cx);
      if (wx == 0.0) continue;
      const int64_t fi = ch.fop + (int64_t)fy * (fnx + 1) + fx;
      const double wi = wx * wy;
      const double mi0 = mask[fi * 2], mi1 = mask[fi * 2 + 1];
      for (int k = 0; k < 9; ++k) {
        const int jx = fx + k % 3 - 1, jy = fy + k / 3 - 1;
        if (jx < 0 || jx > fnx || jy < 0 || jy > fny) continue;
        const int64_t fj = ch.fop + (int64_t)jy * (fnx + 1) + jx;
        const double mj0 = mask[fj * 2], mj1 = mask[fj * 2 + 1];
        const double* a = A + fi * 36 + k * 4;
        const double a00 = wi * mi0 * a[0] * mj0, a01 = wi * mi0 * a[1] * mj1;
        const double a10 = wi * mi1 * a[2] * mj0, a11 = wi * mi1 * a[3] * mj1;
        int px0, px1, py0, py1;
        double vx0, vx1, vy0, vy1;
        parents1d(jx, fnx, px0, vx0, px1, vx1);
        parents1d(jy, fny, py0, vy0, py1, vy1);
        for (int b = 0; b < 2; ++b) {
          const int py = b == 0 ? py0 : py1;
          const double vy = b == 0 ? vy0 : vy1;
          if (py < 0) continue;
          for (int a2 = 0; a2 < 2; ++a2) {
            const int px = a2 == 0 ? px0 : px1;
            const double vx = a2 == 0 ? vx0 : vx1;
            if (px < 0) continue;
            const int kk = (py - cy + 1) * 3 + (px - cx + 1);
            if (kk < 0 || kk > 8) continue;  // cannot happen: parents lie within one coarse step
            const double w = vx * vy;
            acc[kk][0] += a00 * w;
            acc[kk][1] += a01 * w;
            acc[kk][2] += a10 * w;
            acc[kk][3] += a11 * w;
          }
        }
      }
    }
  }
  const int64_t node = ch.op + n;
  for (int c = 0; c < 2; ++c) {
    const bool live = acc[4][c * 2 + c] != 0.0;
    mask[node * 2 + c] = live ? 1.0 : 0.0;
    if (!live) {
      for (int k = 0; k < 9; ++k) acc[k][c * 2] = acc[k][c * 2 + 1] = 0.0;
      acc[4][c * 2 + c] = 1.0;
    }
  }
  for (int k = 0; k < 9; ++k)
    for (int c = 0; c < 4; ++c) A[node * 36 + k * 4 + c] = acc[k][c];
}

// Dense inverse of the coarsest operator of one instance (one block; the
// grid fits in one chunk): Gauss-Jordan without pivoting (the operator is
// SPD), then symmetrised.
__global__ __launch_bounds__(MGB) void k_mg_coarse_setup(const MgChunk* __restrict__ chunks,
                                                         const double* __restrict__ A, double* __restrict__ dense) {
  const MgChunk ch = chunks[blockIdx.x];
  const int N = ch.node_end - ch.node_begin;  // the whole grid
  const int nx = ch.nx;
  const int n = 2 * N;
  double* W = dense + ch.dense_off;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) W[idx] = 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int ix = i % (nx + 1), iy = i / (nx + 1);
    for (int k = 0; k < 9; ++k) {
      const int jx = ix + k % 3 - 1, jy = iy + k / 3 - 1;
      if (jx < 0 || jx > nx || jy < 0 || jy > ch.ny) continue;
      const int j = jy * (nx + 1) + jx;
      for (int c = 0; c < 2; ++c)
        for (int cc = 0; cc < 2; ++cc) W[(2 * i + c) * n + 2 * j + cc] = A[(ch.op + i) * 36 + k * 4 + c * 2 + cc];
    }
  }
  __shared__ double piv;
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    if (threadIdx.x == 0) piv = W[k * n + k];
    __syncthreads();
    const double p = piv;
    for (int j = threadIdx.x; j < n; j += blockDim.x) W[k * n + j] = (j == k ? 1.0 : W[k * n + j]) / p;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      if (i == k) continue;
      const double f = W[i * n + k];
      for (int j = 0; j < n; ++j) W[i * n + j] = (j == k ? 0.0 : W[i * n + j]) - f * W[k * n + j];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    if (i < j) {
      const double v = 0.5 * (W[i * n + j] + W[j * n + i]);
      W[i * n + j] = v;
      W[j * n + i] = v;
    }
  }
}

// Level 0 -> 1: t = r - A0 z at the vertex DOFs (A0 z in the slots), injected;
// pre-smoothing of level 1 from zero: e1 = D1^-1 r1.
__global__ __launch_bounds__(MGB) void k_mg_restrict0(const MgChunk* __restrict__ chunks, PcgDev s,
                                                      const int32_t* __restrict__ vfree, const double* __restrict__ dinv,
                                                      double* __restrict__ r1, double* __restrict__ e1) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int64_t node = ch.op + n, v = ch.vec + n;
  for (int c = 0; c < 2; ++c) {
    const int f = vfree[node * 2 + c];
    double t = 0.0;
    if (f >= 0) {
      const double* sl = s.slots + ch.slot_off + 4 * (int64_t)f;  // a vertex DOF owns 4 slots
      t = s.r[ch.dof_off + f] - (((sl[0] + sl[1]) + sl[2]) + sl[3]);
    }
    r1[v * 2 + c] = t;
    e1[v * 2 + c] = dinv[node * 2 + c] * t;
  }
}

// Level l-1 -> l (l >= 2): r_l = P~^T (r - A e) of the finer level; e_l = D^-1 r_l.
__global__ __launch_bounds__(MGB) void k_mg_restrict(const MgChunk* __restrict__ chunks, PcgDev s,
                                                     const double* __restrict__ A, const double* __restrict__ mask,
                                                     const double* __restrict__ dinv, double* __restrict__ r,
                                                     double* __restrict__ e) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int nx = ch.nx, fnx = ch.fnx, fny = ch.fny;
  const int cx = n % (nx + 1), cy = n / (nx + 1);
  double acc0 = 0.0, acc1 = 0.0;
  const int fxc0 = fine_of(cx, fnx), fyc0 = fine_of(cy, fny);
  for (int oy = -1; oy <= 1; ++oy) {
    const int fy = fyc0 + oy;
    if (fy < 0 || fy > fny) continue;
    const double wy = weight1d(fy, fny, cy);
    if (wy == 0.0) continue;
    for (int ox = -1; ox <= 1; ++ox) {
      const int fx = fxc0 + ox;
      if (fx < 0 || fx > fnx) continue;
      const double wx = weight1d(fx, fnx, cx);
      if (wx == 0.0) continue;
      const int64_t fo = (int64_t)fy * (fnx + 1) + fx;
      const int64_t fi = ch.fop + fo, fv = ch.fvec + fo;
      double t0 = r[fv * 2], t1 = r[fv * 2 + 1];
      for (int k = 0; k < 9; ++k) {
        const int jx = fx + k % 3 - 1, jy = fy + k / 3 - 1;
        if (jx < 0 || jx > fnx || jy < 0 || jy > fny) continue;
        const int64_t jv = ch.fvec + (int64_t)jy * (fnx + 1) + jx;
        const double* a = A + fi * 36 + k * 4;
        const double ej0 = e[jv * 2], ej1 = e[jv * 2 + 1];
        t0 -= a[0] * ej0 + a[1] * ej1;
        t1 -= a[2] * ej0 + a[3] * ej1;
      }
      const double w = wx * wy;
      acc0 += w * mask[fi * 2] * t0;
      acc1 += w * mask[fi * 2 + 1] * t1;
    }
  }
  const int64_t node = ch.op + n, v = ch.vec + n;
  r[v * 2] = acc0;
  r[v * 2 + 1] = acc1;
  e[v * 2] = dinv[node * 2] * acc0;
  e[v * 2 + 1] = dinv[node * 2 + 1] * acc1;
}

// Coarsest level: e2 = A^-1 r (one block per system).
__global__ __launch_bounds__(MGB) void k_mg_coarse_solve(const MgChunk* __restrict__ chunks, PcgDev s,
                                                         const double* __restrict__ dense,
                                                         const double* __restrict__ r, double* __restrict__ e2) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = 2 * (ch.node_end - ch.node_begin);
  const double* W = dense + ch.dense_off;
  const double* rv = r + ch.vec * 2;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(W[i * n + j], rv[j], acc);
    e2[ch.vec * 2 + i] = acc;
  }
}

// Level l (>= 1) going up: e~ = e + P~ e2_coarse, then one l1-Jacobi sweep
// e2 = e~ + D^-1 (r - A e~).
__global__ __launch_bounds__(MGB) void k_mg_prolong_smooth(const MgChunk* __restrict__ chunks, PcgDev s,
                                                           const double* __restrict__ A,
                                                           const double* __restrict__ mask,
                                                           const double* __restrict__ dinv,
                                                           const double* __restrict__ r, const double* __restrict__ e,
                                                           double* __restrict__ e2) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int nx = ch.nx, ny = ch.ny, cnx = ch.cnx;
  const int ix = n % (nx + 1), iy = n / (nx + 1);
  double et[9][2];
  for (int k = 0; k < 9; ++k) {
    const int jx = ix + k % 3 - 1, jy = iy + k / 3 - 1;
    et[k][0] = et[k][1] = 0.0;
    if (jx < 0 || jx > nx || jy < 0 || jy > ny) continue;
    const int64_t jo = (int64_t)jy * (nx + 1) + jx;
    int px0, px1, py0, py1;
    double vx0, vx1, vy0, vy1;
    parents1d(jx, nx, px0, vx0, px1, vx1);
    parents1d(jy, ny, py0, vy0, py1, vy1);
    double c0 = 0.0, c1 = 0.0;
    for (int b = 0; b < 2; ++b) {
      const int py = b == 0 ? py0 : py1;
      const double vy = b == 0 ? vy0 : vy1;
      if (py < 0) continue;
      for (int a2 = 0; a2 < 2; ++a2) {
        const int px = a2 == 0 ? px0 : px1;
        const double vx = a2 == 0 ? vx0 : vx1;
        if (px < 0) continue;
        const int64_t cv = ch.cvec + (int64_t)py * (cnx + 1) + px;
        c0 += vx * vy * e2[cv * 2];
        c1 += vx * vy * e2[cv * 2 + 1];
      }
    }
    const int64_t jn = ch.op + jo, jv = ch.vec + jo;
    et[k][0] = e[jv * 2] + mask[jn * 2] * c0;
    et[k][1] = e[jv * 2 + 1] + mask[jn * 2 + 1] * c1;
  }
  const int64_t node = ch.op + n, v = ch.vec + n;
  double t0 = r[v * 2], t1 = r[v * 2 + 1];
  for (int k = 0; k < 9; ++k) {
    const double* a = A + node * 36 + k * 4;
    t0 -= a[0] * et[k][0] + a[1] * et[k][1];
    t1 -= a[2] * et[k][0] + a[3] * et[k][1];
  }
  e2[v * 2] = et[4][0] + dinv[node * 2] * t0;
  e2[v * 2 + 1] = et[4][1] + dinv[node * 2 + 1] * t1;
}

// Level 1 -> 0: z += injection^T e2_1 at the free vertex DOFs.
__global__ __launch_bounds__(MGB) void k_mg_prolong0(const MgChunk* __restrict__ chunks, PcgDev s,
                                                     const int32_t* __restrict__ vfree, const double* __restrict__ e2) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int64_t node = ch.op + n, v = ch.vec + n;
  for (int c = 0; c < 2; ++c) {
    const int f = vfree[node * 2 + c];
    if (f >= 0) s.z[ch.dof_off + f] += e2[v * 2 + c];
  }
}

// Level-0 post-smoothing z += D0^-1 (r - A0 z) (A0 z in the slots) and the
// partial sums of r.z for the next PCG iteration (parity slot).
__global__ __launch_bounds__(1024) void k_mg_post0(PcgDev s, int it_k, int init) {
  __shared__ double lds[20];
  const Chunk ch = s.chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int par = init ? 0 : ((*s.it_base + it_k + 1) & 1);
  const int64_t o = ch.dof_off;
  double arz = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += blockDim.x) {
    int64_t base;
    int cnt;
    if (i < ch.nfv) {
      base = 4 * (int64_t)i;
      cnt = 4;
    } else if (i < ch.nfv + ch.nfe) {
      base = 4 * (int64_t)ch.nfv + 2 * (int64_t)(i - ch.nfv);
      cnt = 2;
    } else {
      base = 4 * (int64_t)ch.nfv + 2 * (int64_t)ch.nfe + (i - ch.nfv - ch.nfe);
      cnt = 1;
    }
    const double* sl = s.slots + ch.slot_off + base;
    double q = sl[0];
    for (int k = 1; k < cnt; ++k) q += sl[k];
    const double ri = s.r[o + i];
    const double zi = s.z[o + i] + s.dinv[ch.inst_free_off + i] * (ri - q);
    s.z[o + i] = zi;
    arz = fma(ri, zi, arz);
  }
  for (int m = 32; m >= 1; m >>= 1) arz += __shfl_xor(arz, m);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) lds[wave] = arz;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lds[w];
    s.part_rz[par * s.n_chunks + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Element-block additive Schwarz smoother for the hierarchic level.
//
// Point smoothers fail on this level once p >= 2 meets density contrast
// inside an element: the near-null modes of a partly void element are
// combinations of many of its edge and interior modes, which neither a
// diagonal nor the vertex grid below captures.  Each block here is the
// assembled operator restricted to all DOFs of one element, i.e. the
// element's own sum_s E_s K_s plus, on the DOFs it shares, the entries of
// its neighbours, inverted exactly once per design.  The smoother applies
// omega * sum_e P_e^T B_e P_e.  Two elements whose blocks couple through K
// lie within two elements of each other in both directions, so nine colours
// separate the blocks and lambda_max(B K) <= 9: any omega < 2/9 gives a
// convergent, symmetric smoother and keeps the V-cycle SPD.

namespace {
constexpr int ASM_BLOCK = 256;
}

template <int P>
__global__ __launch_bounds__(ASM_BLOCK) void k_asm_block(const GroupDev* __restrict__ groups, int gi,
                                                         const int32_t* __restrict__ nbr,
                                                         const int32_t* __restrict__ el_group,
                                                         const int32_t* __restrict__ el_col,
                                                         const double* __restrict__ E, double* __restrict__ binv) {
  constexpr int NE = ne_of(P);
  constexpr int NEMAX = ne_of(MTO_MAX_P);
  __shared__ double A[NE][NE + 1];
  __shared__ double fcol[NE];
  __shared__ double sc[NE];
  __shared__ int gid[NE];
  __shared__ int pos[NEMAX];
  const GroupDev g = groups[gi];
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  for (int a = tid; a < NE; a += ASM_BLOCK) gid[a] = g.gidx[a * g.npad + k];
  const int cell = g.cell[k];
  for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
    const int a = idx / NE, b = idx - a * NE;
    double v = 0.0;
    for (int sc_ = 0; sc_ < g.S; ++sc_) v = fma(E[cell + sc_], g.ks[((int64_t)sc_ * NE + a) * NE + b], v);
    A[a][b] = v;
  }
  __syncthreads();
  // neighbours: add their entries on pairs of shared DOFs (matched by free index)
  for (int m = 0; m < 8; ++m) {
    const int ge = nbr[m * g.npad + k];
    if (ge < 0) continue;  // uniform over the block
    const GroupDev& gn = groups[el_group[ge]];
    const int kn = el_col[ge];
    const int nen = ne_of(gn.p);
    for (int b = tid; b < nen; b += ASM_BLOCK) {
      const int id = gn.gidx[b * gn.npad + kn];
      int ps = -1;
      if (id >= 0)
        for (int a = 0; a < NE; ++a)
          if (gid[a] == id) {
            ps = a;
            break;
          }
      pos[b] = ps;
    }
    __syncthreads();
    const int celln = gn.cell[kn];
    for (int idx = tid; idx < nen * nen; idx += ASM_BLOCK) {
      const int a = idx / nen, b = idx - a * nen;
      const int pa = pos[a], pb = pos[b];
      if (pa < 0 || pb < 0) continue;
      double v = 0.0;
      for (int sc_ = 0; sc_ < gn.S; ++sc_) v = fma(E[celln + sc_], gn.ks[((int64_t)sc_ * nen + a) * nen + b], v);
      A[pa][pb] += v;  // (a, b) -> (pa, pb) is one-to-one within a neighbour
    }
    __syncthreads();
  }
  // absent or supported DOFs, and DOFs with no stiffness at all (E_min = 0
  // around them): identity rows, zero in the result; then symmetric scaling
  for (int a = tid; a < NE; a += ASM_BLOCK)
    if (!(A[a][a] > 0.0)) gid[a] = -1;
  __syncthreads();
  for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
    const int a = idx / NE, b = idx - a * NE;
    if (gid[a] < 0 || gid[b] < 0) A[a][b] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int a = tid; a < NE; a += ASM_BLOCK) sc[a] = 1.0 / sqrt(A[a][a]);
  __syncthreads();
  for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
    const int a = idx / NE, b = idx - a * NE;
    A[a][b] *= sc[a] * sc[b];
  }
  __syncthreads();
  // Gauss-Jordan inverse in place, no pivoting (the block is SPD)
  for (int kk = 0; kk < NE; ++kk) {
    const double piv = A[kk][kk];
    __syncthreads();
    for (int j = tid; j < NE; j += ASM_BLOCK) A[kk][j] = (j == kk ? 1.0 : A[kk][j]) / piv;
    __syncthreads();
    for (int i = tid; i < NE; i += ASM_BLOCK) fcol[i] = i == kk ? 0.0 : A[i][kk];
    __syncthreads();
    for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
      const int i = idx / NE, j = idx - i * NE;
      if (i != kk) A[i][j] = (j == kk ? 0.0 : A[i][j]) - fcol[i] * A[kk][j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
    const int a = idx / NE, b = idx - a * NE;
    double v = 0.5 * (A[a][b] + A[b][a]) * sc[a] * sc[b];
    if (gid[a] < 0 || gid[b] < 0) v = 0.0;
    binv[(int64_t)idx * g.npad + k] = v;
  }
}

// slots = omega * B_e v_e: one wave per tile, 16 element columns at a time;
// lane = (row quarter, column).
template <int P>
__global__ __launch_bounds__(64) void k_asm_apply(GroupDev g, const Tile* __restrict__ tiles,
                                                  const double* __restrict__ binv, const double* __restrict__ v,
                                                  PcgDev s, double omega) {
  constexpr int NE = ne_of(P);
  __shared__ double vs[NE][17];
  const Tile t = tiles[g.tile_begin + blockIdx.x];
  if (s.status[t.sys] != SYS_RUNNING) return;
  const int lane = threadIdx.x, c = lane & 15, qd = lane >> 4;
  const double* __restrict__ vsys = v + t.dof_off;
  double* __restrict__ sl = s.slots + t.slot_off;
  for (int c0 = 0; c0 < t.count; c0 += 16) {
    const bool valid = c0 + c < t.count;
    const int col = t.elem_begin + c0 + (valid ? c : 0);
    for (int r = qd; r < NE; r += 4) {
      const int id = valid ? g.gidx[r * g.npad + col] : -1;
      vs[r][c] = id >= 0 ? vsys[id] : 0.0;
    }
    __syncthreads();
    for (int a = qd; a < NE; a += 4) {
      const double* __restrict__ bp = binv + (int64_t)a * NE * g.npad + col;
      double acc = 0.0;
#pragma unroll 10
      for (int b = 0; b < NE; ++b) acc = fma(bp[(int64_t)b * g.npad], vs[b][c], acc);
      const int si = valid ? g.sidx[a * g.npad + col] : -1;
      if (si >= 0) sl[si] = omega * acc;
    }
    __syncthreads();
  }
}

// z = assembled slots
__global__ __launch_bounds__(1024) void k_asm_z(PcgDev s) {
  const Chunk ch = s.chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int i = ch.begin + threadIdx.x;
  if (i >= ch.end) return;
  s.z[ch.dof_off + i] = slot_sum(s.slots + ch.slot_off, i, ch.nfv, ch.nfe);
}

// q = r - assembled slots
__global__ __launch_bounds__(1024) void k_asm_resid(PcgDev s) {
  const Chunk ch = s.chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int i = ch.begin + threadIdx.x;
  if (i >= ch.end) return;
  const int64_t o = ch.dof_off + i;
  s.q[o] = s.r[o] - slot_sum(s.slots + ch.slot_off, i, ch.nfv, ch.nfe);
}

// z += assembled slots; partial sums of r.z for the next PCG iteration
__global__ __launch_bounds__(1024) void k_asm_post(PcgDev s, int it_k, int init) {
  __shared__ double lds[20];
  const Chunk ch = s.chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int par = init ? 0 : ((*s.it_base + it_k + 1) & 1);
  const int i = ch.begin + threadIdx.x;
  double arz = 0.0;
  if (i < ch.end) {
    const int64_t o = ch.dof_off + i;
    const double zi = s.z[o] + slot_sum(s.slots + ch.slot_off, i, ch.nfv, ch.nfe);
    s.z[o] = zi;
    arz = s.r[o] * zi;
  }
  for (int m = 32; m >= 1; m >>= 1) arz += __shfl_xor(arz, m);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) lds[wave] = arz;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lds[w];
    s.part_rz[par * s.n_chunks + blockIdx.x] = t;
  }
}

// ---- launchers ----
void launch_mg_assemble1(const MgChunk* ch, int n, const MgElem* elems, const double* kv, const double* E,
                         const int32_t* vfree, double* A, double* mask, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_assemble1, dim3(n), dim3(MGB), 0, st, ch, elems, kv, E, vfree, A, mask);
}
void launch_mg_l1(const MgChunk* ch, int n, const double* A, double* dinv, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_l1, dim3(n), dim3(MGB), 0, st, ch, A, dinv);
}
void launch_mg_rap(const MgChunk* ch, int n, double* A, double* mask, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_rap, dim3(n), dim3(MGB), 0, st, ch, A, mask);
}
void launch_mg_coarse_setup(const MgChunk* ch, int n, const double* A, double* dense, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_coarse_setup, dim3(n), dim3(MGB), 0, st, ch, A, dense);
}
void launch_mg_restrict0(const MgChunk* ch, int n, const PcgDev& s, const int32_t* vfree, const double* dinv,
                         double* r1, double* e1, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_restrict0, dim3(n), dim3(MGB), 0, st, ch, s, vfree, dinv, r1, e1);
}
void launch_mg_restrict(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* mask,
                        const double* dinv, double* r, double* e, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_restrict, dim3(n), dim3(MGB), 0, st, ch, s, A, mask, dinv, r, e);
}
void launch_mg_coarse_solve(const MgChunk* ch, int n, const PcgDev& s, const double* dense, const double* r,
                            double* e2, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_coarse_solve, dim3(n), dim3(MGB), 0, st, ch, s, dense, r, e2);
}
void launch_mg_prolong_smooth(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* mask,
                              const double* dinv, const double* r, const double* e, double* e2, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_prolong_smooth, dim3(n), dim3(MGB), 0, st, ch, s, A, mask, dinv, r, e, e2);
}
void launch_mg_prolong0(const MgChunk* ch, int n, const PcgDev& s, const int32_t* vfree, const double* e2,
                        hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_prolong0, dim3(n), dim3(MGB), 0, st, ch, s, vfree, e2);
}
void launch_mg_post0(const PcgDev& s, int it_k, int init, hipStream_t st) {
  hipLaunchKernelGGL(k_mg_post0, dim3(s.n_chunks), dim3(1024), 0, st, s, it_k, init);
}

void launch_asm_block(const GroupDev& g, int gi, const GroupDev* groups, const int32_t* nbr, const int32_t* el_group,
                      const int32_t* el_col, const double* E, double* binv, hipStream_t st) {
  if (g.n_elems == 0) return;
  const dim3 grid(g.n_elems), block(ASM_BLOCK);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_asm_block<1>, grid, block, 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
    case 2: hipLaunchKernelGGL(k_asm_block<2>, grid, block, 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
    case 3: hipLaunchKernelGGL(k_asm_block<3>, grid, block, 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
    default: hipLaunchKernelGGL(k_asm_block<4>, grid, block, 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
  }
}
void launch_asm_apply(const GroupDev& g, const Tile* tiles, const double* binv, const double* v, const PcgDev& s,
                      double omega, hipStream_t st) {
  if (g.n_tiles == 0) return;
  const dim3 grid(g.n_tiles), block(64);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_asm_apply<1>, grid, block, 0, st, g, tiles, binv, v, s, omega); break;
    case 2: hipLaunchKernelGGL(k_asm_apply<2>, grid, block, 0, st, g, tiles, binv, v, s, omega); break;
    case 3: hipLaunchKernelGGL(k_asm_apply<3>, grid, block, 0, st, g, tiles, binv, v, s, omega); break;
    default: hipLaunchKernelGGL(k_asm_apply<4>, grid, block, 0, st, g, tiles, binv, v, s, omega); break;
  }
}
void launch_asm_z(const PcgDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_asm_z, dim3(s.n_chunks), dim3(1024), 0, st, s);
}
void launch_asm_resid(const PcgDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_asm_resid, dim3(s.n_chunks), dim3(1024), 0, st, s);
}
void launch_asm_post(const PcgDev& s, int it_k, int init, hipStream_t st) {
  hipLaunchKernelGGL(k_asm_post, dim3(s.n_chunks), dim3(1024), 0, st, s, it_k, init);
}


}  // namespace mto
