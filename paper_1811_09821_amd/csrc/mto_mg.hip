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

// ---- the coarsest level: dense inverse from a banded Cholesky factor ----
//
// The coarsest grid (up to MG_COARSE_MAX DOFs) is solved exactly by a dense
// inverse, formed once per design: its DOFs are renumbered with the shorter
// side of the grid running fastest, which makes the operator banded with
// lower bandwidth b = 2 m + 5 (m elements along the short side); a
// right-looking band Cholesky runs in one block with a sliding window of
// b + 1 rows in LDS; then every column of the inverse is one forward and one
// backward band substitution, one thread per column; finally symmetrised.

// node q couples to q +- (m + 2) at most (m = elements along the short side),
// so DOF 2 q + c couples to DOFs at most 2 (m + 2) + 1 away
__device__ __forceinline__ int band_width(const MgChunk& ch) { return 2 * min(ch.nx, ch.ny) + 5; }

// node of band position q (the shorter side runs fastest)
__device__ __forceinline__ void band_node(const MgChunk& ch, int q, int& ix, int& iy) {
  if (ch.ny <= ch.nx) {
    ix = q / (ch.ny + 1);
    iy = q - ix * (ch.ny + 1);
  } else {
    iy = q / (ch.nx + 1);
    ix = q - iy * (ch.nx + 1);
  }
}

// entry (d1, d2) of the coarsest operator in band numbering (DOF 2 q + c)
__device__ __forceinline__ double band_entry(const MgChunk& ch, const double* __restrict__ A, int d1, int d2) {
  int x1, y1, x2, y2;
  band_node(ch, d1 >> 1, x1, y1);
  band_node(ch, d2 >> 1, x2, y2);
  const int dx = x2 - x1, dy = y2 - y1;
  if (dx < -1 || dx > 1 || dy < -1 || dy > 1) return 0.0;
  const int64_t node = ch.op + (int64_t)y1 * (ch.nx + 1) + x1;
  return A[node * 36 + ((dy + 1) * 3 + (dx + 1)) * 4 + (d1 & 1) * 2 + (d2 & 1)];
}

// Band Cholesky of one instance's coarsest operator: band[j][k] = L[j][j - k].
// Two barriers per column: (1) scale column j below the diagonal and retire
// row j to global memory; (2) the rank-1 update of the window and the load of
// row j + b + 1 into the slot row j has left.
__global__ __launch_bounds__(1024) void k_mg_coarse_chol(const MgChunk* __restrict__ chunks,
                                                        const double* __restrict__ A, double* __restrict__ band) {
  extern __shared__ double W[];  // window [(b + 1)][(b + 1)], row i in slot i % (b + 1)
  const MgChunk ch = chunks[blockIdx.x];
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int b = band_width(ch), w = b + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* __restrict__ out = band + ch.band_off;
  for (int idx = tid; idx < w * w; idx += nt) {
    const int r = idx / w, k = idx - r * w;
    W[idx] = (r < n && r - k >= 0) ? band_entry(ch, A, r, r - k) : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int sj = j % w;
    const double d = sqrt(W[sj * w]);
    const int m = min(b, n - 1 - j);
    for (int ii = tid; ii < m; ii += nt) {
      const int i = j + 1 + ii;
      W[(i % w) * w + (i - j)] /= d;
    }
    for (int k = tid; k < w; k += nt) out[(int64_t)j * w + k] = k == 0 ? d : W[sj * w + k];
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += nt) {
      const int ii = idx / m, kk = idx - ii * m;
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      W[(i % w) * w + (i - k)] -= W[(i % w) * w + (i - j)] * W[(k % w) * w + (k - j)];
    }
    const int r = j + w;  // first touched by step j + 1
    for (int k = tid; k < w; k += nt) W[sj * w + k] = (r < n && r - k >= 0) ? band_entry(ch, A, r, r - k) : 0.0;
    __syncthreads();
  }
}

// Column c of the inverse (band numbering) per wave: y = L^-1 e_c, then
// x = L^-T y, held in LDS; each substitution step is a band dot product
// spread over the 64 lanes.  Stored as row c (the inverse is symmetric, and
// rows are contiguous).
constexpr int MG_INV_WAVES = 2;

__global__ __launch_bounds__(64 * MG_INV_WAVES) void k_mg_coarse_inv(const MgChunk* __restrict__ chunks,
                                                                     const double* __restrict__ band,
                                                                     double* __restrict__ dense, int nmax) {
  extern __shared__ double xs_all[];  // [MG_INV_WAVES][nmax]
  const MgChunk ch = chunks[blockIdx.y];
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * MG_INV_WAVES + wave;
  if (c >= n) return;  // whole wave
  const int b = band_width(ch), w = b + 1;
  const double* __restrict__ L = band + ch.band_off;
  double* xs = xs_all + wave * nmax;
  for (int i = lane; i < n; i += 64) xs[i] = 0.0;
  // forward: rows c .. n-1 (y_i = 0 above c)
  for (int i = c; i < n; ++i) {
    double acc = 0.0;
    for (int k = i - 1 - lane; k >= max(c, i - b); k -= 64) acc = fma(L[(int64_t)i * w + (i - k)], xs[k], acc);
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    const double yi = ((i == c ? 1.0 : 0.0) - acc) / L[(int64_t)i * w];
    if (lane == 0) xs[i] = yi;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  // backward: rows n-1 .. 0
  for (int i = n - 1; i >= 0; --i) {
    double acc = 0.0;
    const int kend = min(n - 1, i + b);
    for (int k = i + 1 + lane; k <= kend; k += 64) acc = fma(L[(int64_t)k * w + (k - i)], xs[k], acc);
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    const double xi = (xs[i] - acc) / L[(int64_t)i * w];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) xs[i] = xi;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  double* __restrict__ X = dense + ch.dense_off + (int64_t)c * n;
  for (int i = lane; i < n; i += 64) X[i] = xs[i];
}

// X = (X + X^T) / 2
__global__ __launch_bounds__(256) void k_mg_coarse_sym(const MgChunk* __restrict__ chunks, double* __restrict__ dense) {
  const MgChunk ch = chunks[blockIdx.y];
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
  if (j <= i) return;
  double* __restrict__ X = dense + ch.dense_off;
  const double v = 0.5 * (X[(int64_t)i * n + j] + X[(int64_t)j * n + i]);
  X[(int64_t)i * n + j] = v;
  X[(int64_t)j * n + i] = v;
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

// ---- per-node steps of levels >= 1 (shared by the one-level kernels and
// the fused coarse cycle) ----

// Residual of a level after its pre-smoothing: t = r - A e.
__device__ __forceinline__ void mg_resid_node(const MgChunk& ch, int n, const double* __restrict__ A,
                                              const double* __restrict__ r, const double* __restrict__ e,
                                              double* __restrict__ t) {
  const int nx = ch.nx, ny = ch.ny;
  const int ix = n % (nx + 1), iy = n / (nx + 1);
  const int64_t node = ch.op + n, v = ch.vec + n;
  double t0 = r[v * 2], t1 = r[v * 2 + 1];
  for (int k = 0; k < 9; ++k) {
    const int jx = ix + k % 3 - 1, jy = iy + k / 3 - 1;
    if (jx < 0 || jx > nx || jy < 0 || jy > ny) continue;
    const int64_t jv = ch.vec + (int64_t)jy * (nx + 1) + jx;
    const double* a = A + node * 36 + k * 4;
    const double ej0 = e[jv * 2], ej1 = e[jv * 2 + 1];
    t0 -= a[0] * ej0 + a[1] * ej1;
    t1 -= a[2] * ej0 + a[3] * ej1;
  }
  t[v * 2] = t0;
  t[v * 2 + 1] = t1;
}

// Restriction to this level: r = P~^T t of the finer level's residual, and
// the pre-smoothing from zero e = D^-1 r.
__device__ __forceinline__ void mg_restrict_node(const MgChunk& ch, int n, const double* __restrict__ mask,
                                                 const double* __restrict__ dinv, const double* __restrict__ t,
                                                 double* __restrict__ r, double* __restrict__ e) {
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
      const double w = wx * wy;
      acc0 += w * mask[fi * 2] * t[fv * 2];
      acc1 += w * mask[fi * 2 + 1] * t[fv * 2 + 1];
    }
  }
  const int64_t node = ch.op + n, v = ch.vec + n;
  r[v * 2] = acc0;
  r[v * 2 + 1] = acc1;
  e[v * 2] = dinv[node * 2] * acc0;
  e[v * 2 + 1] = dinv[node * 2 + 1] * acc1;
}

// Going up: e~ = e + P~ e2_coarse, then one l1-Jacobi sweep
// e2 = e~ + D^-1 (r - A e~).
__device__ __forceinline__ void mg_prolong_smooth_node(const MgChunk& ch, int n, const double* __restrict__ A,
                                                       const double* __restrict__ mask,
                                                       const double* __restrict__ dinv,
                                                       const double* __restrict__ r, const double* __restrict__ e,
                                                       double* __restrict__ e2) {
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

__global__ __launch_bounds__(MGB) void k_mg_resid(const MgChunk* __restrict__ chunks, PcgDev s,
                                                  const double* __restrict__ A, const double* __restrict__ r,
                                                  const double* __restrict__ e, double* __restrict__ t) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n < ch.node_end) mg_resid_node(ch, n, A, r, e, t);
}

__global__ __launch_bounds__(MGB) void k_mg_restrict(const MgChunk* __restrict__ chunks, PcgDev s,
                                                     const double* __restrict__ mask, const double* __restrict__ dinv,
                                                     const double* __restrict__ t, double* __restrict__ r,
                                                     double* __restrict__ e) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n < ch.node_end) mg_restrict_node(ch, n, mask, dinv, t, r, e);
}

// Coarsest level: e2 = X r with the dense inverse X (band numbering, so r
// and e2 are permuted on the way).  Grid (row blocks of 16, systems); 16
// lanes per row read contiguous stretches of the row.
__global__ __launch_bounds__(256) void k_mg_coarse_solve(const MgChunk* __restrict__ chunks, PcgDev s,
                                                         const double* __restrict__ dense,
                                                         const double* __restrict__ r, double* __restrict__ e2) {
  const MgChunk ch = chunks[blockIdx.y];
  if (!sys_running(s, ch.sys)) return;
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int i = blockIdx.x * 16 + (threadIdx.x >> 4), l16 = threadIdx.x & 15;
  const bool row_ok = i < n;
  const double* __restrict__ X = dense + ch.dense_off + (int64_t)(row_ok ? i : 0) * n;
  double acc = 0.0;
  if (row_ok)
    for (int j = l16; j < n; j += 16) {
      int x, y;
      band_node(ch, j >> 1, x, y);
      acc = fma(X[j], r[(ch.vec + (int64_t)y * (ch.nx + 1) + x) * 2 + (j & 1)], acc);
    }
  for (int m = 8; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
  if (row_ok && l16 == 0) {
    int x, y;
    band_node(ch, i >> 1, x, y);
    e2[(ch.vec + (int64_t)y * (ch.nx + 1) + x) * 2 + (i & 1)] = acc;
  }
}

__global__ __launch_bounds__(MGB) void k_mg_prolong_smooth(const MgChunk* __restrict__ chunks, PcgDev s,
                                                           const double* __restrict__ A,
                                                           const double* __restrict__ mask,
                                                           const double* __restrict__ dinv,
                                                           const double* __restrict__ r, const double* __restrict__ e,
                                                           double* __restrict__ e2) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n < ch.node_end) mg_prolong_smooth_node(ch, n, A, mask, dinv, r, e, e2);
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
constexpr int ASM_APPLY_BLOCK = 256;

// Position of (a, b), a <= b, in the row-packed upper triangle of an NE x NE matrix.
template <int NE>
__device__ __forceinline__ int packed_index(int a, int b) {
  return a * NE - (a * (a - 1)) / 2 + (b - a);
}
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
  // upper triangle, packed by rows (the inverse is symmetric)
  for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
    const int a = idx / NE, b = idx - a * NE;
    if (b < a) continue;
    double v = 0.5 * (A[a][b] + A[b][a]) * sc[a] * sc[b];
    if (gid[a] < 0 || gid[b] < 0) v = 0.0;
    binv[(int64_t)packed_index<NE>(a, b) * g.npad + k] = v;
  }
}

// slots = omega * B_e v_e: one block per tile, 16 element columns at a time;
// thread = (row group, column), rows rg, rg + 16, ...  B_e is read from the
// packed upper triangle (row a takes entry (min(a, b), max(a, b))).
template <int P>
__global__ __launch_bounds__(ASM_APPLY_BLOCK) void k_asm_apply(GroupDev g, const Tile* __restrict__ tiles,
                                                               const double* __restrict__ binv,
                                                               const double* __restrict__ v, PcgDev s,
                                                               double omega) {
  constexpr int NE = ne_of(P);
  __shared__ double vs[NE][17];
  const Tile t = tiles[g.tile_begin + blockIdx.x];
  if (s.status[t.sys] != SYS_RUNNING) return;
  const int c = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const double* __restrict__ vsys = v + t.dof_off;
  double* __restrict__ sl = s.slots + t.slot_off;
  const int64_t np = g.npad;
  for (int c0 = 0; c0 < t.count; c0 += 16) {
    const bool valid = c0 + c < t.count;
    const int col = t.elem_begin + c0 + (valid ? c : 0);
    for (int r = rg; r < NE; r += 16) {
      const int id = valid ? g.gidx[r * np + col] : -1;
      vs[r][c] = id >= 0 ? vsys[id] : 0.0;
    }
    __syncthreads();
    for (int a = rg; a < NE; a += 16) {
      const double* __restrict__ bp = binv + col;
      double acc = 0.0;
      for (int b = 0; b < a; ++b) acc = fma(bp[packed_index<NE>(b, a) * np], vs[b][c], acc);
      const double* __restrict__ row = bp + (int64_t)packed_index<NE>(a, a) * np;
#pragma unroll 8
      for (int b = a; b < NE; ++b) acc = fma(row[(b - a) * np], vs[b][c], acc);
      const int si = valid ? g.sidx[a * np + col] : -1;
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
void launch_mg_coarse_setup(const MgChunk* ch, int n, int nmax, int bmax, const double* A, double* band, double* dense,
                            hipStream_t st) {
  if (!n) return;
  const size_t lds = (size_t)(bmax + 1) * (bmax + 1) * 8;
  hipLaunchKernelGGL(k_mg_coarse_chol, dim3(n), dim3(1024), lds, st, ch, A, band);
  hipLaunchKernelGGL(k_mg_coarse_inv, dim3((nmax + MG_INV_WAVES - 1) / MG_INV_WAVES, n), dim3(64 * MG_INV_WAVES),
                     (size_t)MG_INV_WAVES * nmax * 8, st, ch, band, dense, nmax);
  const int64_t nn = (int64_t)nmax * nmax;
  hipLaunchKernelGGL(k_mg_coarse_sym, dim3((unsigned)((nn + 255) / 256), n), dim3(256), 0, st, ch, dense);
}
void launch_mg_restrict0(const MgChunk* ch, int n, const PcgDev& s, const int32_t* vfree, const double* dinv,
                         double* r1, double* e1, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_restrict0, dim3(n), dim3(MGB), 0, st, ch, s, vfree, dinv, r1, e1);
}
void launch_mg_resid(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* r, const double* e,
                     double* t, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_resid, dim3(n), dim3(MGB), 0, st, ch, s, A, r, e, t);
}
void launch_mg_restrict(const MgChunk* ch, int n, const PcgDev& s, const double* mask, const double* dinv,
                        const double* t, double* r, double* e, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_restrict, dim3(n), dim3(MGB), 0, st, ch, s, mask, dinv, t, r, e);
}
void launch_mg_coarse_solve(const MgChunk* ch, int n, int nmax, const PcgDev& s, const double* dense, const double* r,
                            double* e2, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_coarse_solve, dim3((nmax + 15) / 16, n), dim3(256), 0, st, ch, s, dense, r, e2);
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
  const dim3 grid(g.n_tiles), block(ASM_APPLY_BLOCK);
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
