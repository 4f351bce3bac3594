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

#include <algorithm>
#include <cstdlib>
#include <type_traits>

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
#pragma unroll
  for (int oy = -1; oy <= 1; ++oy) {
    const int fy = fyc0 + oy;
    if (fy < 0 || fy > fny) continue;
    const double wy = weight1d(fy, fny, cy);
    if (wy == 0.0) continue;
#pragma unroll
    for (int ox = -1; ox <= 1; ++ox) {
      const int fx = fxc0 + ox;
      if (fx < 0 || fx > fnx) continue;
      const double wx = weight1d(fx, fnx, cx);
      if (wx == 0.0) continue;
      const int64_t fi = ch.fop + (int64_t)fy * (fnx + 1) + fx;
      const double wi = wx * wy;
      const double mi0 = mask[fi * 2], mi1 = mask[fi * 2 + 1];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int jx = fx + k % 3 - 1, jy = fy + k / 3 - 1;
        if (jx < 0 || jx > fnx || jy < 0 || jy > fny) continue;
        const int64_t fj = ch.fop + (int64_t)jy * (fnx + 1) + jx;
        const double mj0 = mask[fj * 2], mj1 = mask[fj * 2 + 1];
        const double* a = A + fi * 36 + k * 4;
        const double a00 = wi * mi0 * a[0] * mj0, a01 = wi * mi0 * a[1] * mj1;
        const double a10 = wi * mi1 * a[2] * mj0, a11 = wi * mi1 * a[3] * mj1;
        // weights of fine node j in the coarse nodes around (cx, cy), per axis:
        // its parents lie within one coarse step, so every accumulator index
        // below is a compile-time constant (no private-memory array)
        int px0, px1, py0, py1;
        double vx0, vx1, vy0, vy1;
        parents1d(jx, fnx, px0, vx0, px1, vx1);
        parents1d(jy, fny, py0, vy0, py1, vy1);
        double wxk[3], wyk[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          wxk[d] = (px0 == cx + d - 1 ? vx0 : 0.0) + (px1 == cx + d - 1 ? vx1 : 0.0);
          wyk[d] = (py0 == cy + d - 1 ? vy0 : 0.0) + (py1 == cy + d - 1 ? vy1 : 0.0);
        }
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) {
          const double w = wyk[kk / 3] * wxk[kk % 3];
          acc[kk][0] = fma(a00, w, acc[kk][0]);
          acc[kk][1] = fma(a01, w, acc[kk][1]);
          acc[kk][2] = fma(a10, w, acc[kk][2]);
          acc[kk][3] = fma(a11, w, acc[kk][3]);
        }
      }
    }
  }
  const int64_t node = ch.op + n;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const bool live = acc[4][c * 2 + c] != 0.0;
    mask[node * 2 + c] = live ? 1.0 : 0.0;
    if (!live) {
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[k][c * 2] = acc[k][c * 2 + 1] = 0.0;
      acc[4][c * 2 + c] = 1.0;
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) A[node * 36 + k * 4 + c] = acc[k][c];
}

// ---- the coarsest level: dense inverse from a banded Cholesky factor ----
//
// The coarsest grid (up to MG_COARSE_MAX DOFs) is solved exactly by a dense
// inverse, formed once per design: its DOFs are renumbered with the shorter
// side of the grid running fastest, which makes the operator banded with
// lower bandwidth b = 2 m + 5 (m elements along the short side); a blocked
// right-looking band Cholesky runs in one block with a sliding window of rows
// in LDS; then every column of the inverse's lower triangle is one forward
// and one (truncated) backward band substitution in one wave; finally the
// triangle is mirrored into the natural numbering.

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

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Blocked band Cholesky of one instance's coarsest operator, NB columns per
// step.  Outputs: the row form (L[i][i - t]) and the column form
// (L[j + 1 + t][j]), each with 1 / L[i][i], in the padded layout described
// with MG_BAND_RS.
//   Window: rows J .. J + b + NB - 1 in a ring of R = b + NB slots (row i in
//   slot i % R), slot row t holding entry (i, i - t).
//   Step J: wave 0 factors the panel (columns J .. J + NB - 1 of its R rows,
//   one or two rows per lane, in registers; diagonal and column entries broadcast
//   with lane reads) and leaves it, with the reciprocal diagonal, in LDS.
//   After a barrier the rank-NB update of the trailing b x b triangle runs
//   on the matrix cores: 16 x 16 tiles of it, one per wave (at most 15), each
//   two v_mfma_f64_16x16x4f64 on panel rows read from LDS.  Meanwhile waves
//   1 .. 11 refill the NB retired slots with the next rows of the operator
//   (loaded before the barrier) and waves 12 .. 15 write the panel to both
//   outputs.  Two barriers per NB columns.  Only the writer waves issue
//   global stores, so no other wave ever waits for their completion.
constexpr int MG_CHOL_BLOCK = 1024;
constexpr int MG_CHOL_NB = 8;
constexpr int MG_CHOL_LP = MG_CHOL_NB + 1;  // panel row stride in LDS (odd, against bank conflicts)

__host__ __device__ constexpr int chol_tiles(int b) {  // 16 x 16 tiles of the trailing triangle
  return ((b + 15) / 16) * ((b + 15) / 16 + 1) / 2;
}
static_assert(chol_tiles(MG_BAND_MAX) <= MG_CHOL_BLOCK / 64 - 1, "one trailing tile per wave 1..");
constexpr int MG_CHOL_WRITER0 = 768;  // first writer thread (waves 12 .. 15)
static_assert(64 + MG_CHOL_NB * (MG_BAND_MAX + 1) <= MG_CHOL_WRITER0, "one refill entry per thread of waves 1 .. 11");
static_assert(MG_CHOL_NB + 16 * ((MG_BAND_MAX + 15) / 16) <= 128, "panel rows must fit two per lane");
static_assert(MG_CHOL_NB == 8, "two MFMA k-steps of 4");

// panel rows kept in LDS: the window's R rows and zero rows up to whole tiles
__host__ __device__ constexpr int chol_panel_rows(int b) { return MG_CHOL_NB + 16 * ((b + 15) / 16); }

size_t chol_lds_bytes(int b) {
  const int R = b + MG_CHOL_NB;
  return (size_t)(R * (b + 1) + chol_panel_rows(b) * MG_CHOL_LP + MG_CHOL_NB) * sizeof(double);
}

typedef double chol_d4 __attribute__((ext_vector_type(4)));
typedef double d4m __attribute__((ext_vector_type(4)));

// Q panel rows per lane of wave 0: 1 when the panel (chol_panel_rows) fits in
// 64 rows, else 2.
template <int Q>
__global__ __launch_bounds__(MG_CHOL_BLOCK) void k_mg_coarse_chol(const MgChunk* __restrict__ chunks,
                                                                 const double* __restrict__ A,
                                                                 double* __restrict__ band) {
  extern __shared__ double lds_chol[];
  constexpr int NB = MG_CHOL_NB, LP = MG_CHOL_LP;
  const MgChunk ch = chunks[blockIdx.x];
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int b = band_width(ch), w = b + 1, R = b + NB, RP = chol_panel_rows(b);
  double* __restrict__ W = lds_chol;            // [R][w]
  double* __restrict__ Lp = lds_chol + R * w;   // [RP][LP]: panel row J + r at r
  double* __restrict__ rjl = Lp + RP * LP;      // [NB]: 1 / L[J + t][J + t]
  const int tid = threadIdx.x, nt = blockDim.x, wave = tid >> 6, lane = tid & 63;
  double* __restrict__ out = band + ch.band_off + MG_INV_PD * MG_BAND_RS;                   // row form
  double* __restrict__ outc = band + ch.band_off + (int64_t)(n + 2 * MG_INV_PD) * MG_BAND_RS;  // column form
  for (int idx = tid; idx < R * w; idx += nt) {
    const int r = idx / w, t = idx - r * w;
    W[idx] = (r < n && r - t >= 0) ? band_entry(ch, A, r, r - t) : 0.0;
  }
  // this wave's trailing tile (rows 16 tI.., columns 16 tK.., tK <= tI), if any
  int tI = -1, tK = 0;
  {
    const int nT = (b + 15) >> 4;
    int k = wave - 1;
    if (k >= 0 && k < nT * (nT + 1) / 2)
      for (int I = 0; I < nT; ++I) {
        if (k <= I) {
          tI = I;
          tK = k;
          break;
        }
        k -= I + 1;
      }
  }
  const int at = tid - 64;                                         // refill entry (waves 1 .. 11)
  const int wt = tid - MG_CHOL_WRITER0, n_wt = nt - MG_CHOL_WRITER0;  // writer index (waves 12 .. 15)
  __syncthreads();
  for (int J = 0; J < n; J += NB) {  // uniform
    const int nb = min(NB, n - J);
    // rows J + R .. J + R + NB - 1 go to the slots of rows J .. J + NB - 1 after the panel
    double pre = 0.0;
    int pre_at = -1;
    if (at >= 0 && tid < MG_CHOL_WRITER0 && at < NB * w) {
      const int r = J + R + at / w, t = at - (at / w) * w;
      pre_at = (r % R) * w + t;
      if (r < n && r - t >= 0) pre = band_entry(ch, A, r, r - t);
    }
    if (wave == 0) {
      double p[Q][NB];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int r = lane + 64 * q, i = J + r;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const int o = r - t;
          p[q][t] = (r < R && i < n && o >= 0 && o <= b) ? W[(i % R) * w + o] : 0.0;
        }
      }
      double rjs = 0.0;  // lane t < NB keeps 1 / L[J + t][J + t]
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t >= nb) break;  // uniform
        // 1 / sqrt(d): the hardware estimate refined by two Newton steps
        // y <- y (3/2 - d y^2 / 2), each squaring its relative error; then
        // L_jj = d / sqrt(d).  Shorter than a rounded sqrt and a division.
        const double d = readlane_f64(p[0][t], t), hd = 0.5 * d;
        double rj = __builtin_amdgcn_rsq(d);
        rj *= fma(-hd * rj, rj, 1.5);
        rj *= fma(-hd * rj, rj, 1.5);
        const double dj = d * rj;
        if (lane == t) rjs = rj;
        // rows above the diagonal are zeroed here (rows 64.. are all below)
        p[0][t] = lane > t ? p[0][t] * rj : (lane == t ? dj : 0.0);
        if (Q == 2) p[Q - 1][t] *= rj;
        // Unpredicated: a row r < t2 takes garbage in its (upper) column t2,
        // which the scaling of column t2 zeroes before anything reads it.
#pragma unroll
        for (int t2 = t + 1; t2 < NB; ++t2) {
          const double v = readlane_f64(p[0][t], t2);  // L[J + t2][J + t]
#pragma unroll
          for (int q = 0; q < Q; ++q) p[q][t2] = fma(-p[q][t], v, p[q][t2]);
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int r = lane + 64 * q;
        if (r < RP) {
#pragma unroll
          for (int t = 0; t < NB; ++t) Lp[r * LP + t] = p[q][t];
        }
      }
      if (lane < NB) rjl[lane] = rjs;
    }
    __syncthreads();
    if (tI >= 0) {
      // A[m][k] = L[J + NB + 16 tI + m][J + k], B[k][c] = L[J + NB + 16 tK + c][J + k]
      const int m = lane & 15, k4 = lane >> 4;
      const double* __restrict__ la = Lp + (NB + 16 * tI + m) * LP + k4;
      const double* __restrict__ lb = Lp + (NB + 16 * tK + m) * LP + k4;
      chol_d4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(la[0], lb[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(la[4], lb[4], acc, 0, 0, 0);
      // D lane l holds D[l / 16 + 4 r][l % 16]
      const int kk = 16 * tK + m;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * tI + k4 + 4 * r, i = J + NB + ii;
        if (kk <= ii && ii < b && i < n) W[(i % R) * w + (ii - kk)] -= acc[r];
      }
    }
    if (pre_at >= 0) W[pre_at] = pre;
    if (wt >= 0) {
      // the panel's entries (J + r, J + t), o = r - t, to both output forms
      for (int e = wt; e < R * NB; e += n_wt) {
        const int r = e / NB, t = e - (e / NB) * NB, i = J + r, o = r - t;
        if (t < nb && i < n && o >= 0 && o <= b) {
          if (o == 0) {
            const double rj = rjl[t];
            out[(int64_t)i * MG_BAND_RS + 128] = rj;
            outc[(int64_t)i * MG_BAND_CS + 127] = rj;
          } else {
            const double v = Lp[r * LP + t];
            out[(int64_t)i * MG_BAND_RS + o] = v;
            outc[(int64_t)(J + t) * MG_BAND_CS + (o - 1)] = v;
          }
        }
      }
    }
    __syncthreads();
  }
}

// Column c of the inverse's lower triangle (band numbering) per wave:
// y = L^-1 e_c (rows c .. n-1), then x = L^-T y for rows n-1 down to c, by
// column-oriented substitution.  Every pending row keeps its running sum in
// the lane congruent to it mod 64: before step i a lane holds its nearest
// row on the unfinished side of i ("near") and the next one beyond ("far",
// 64 further); b < 128 keeps every row of the band in one of the two.  A
// step finishes row i in lane i % 64 (one multiply by 1 / L[i][i], which
// that lane finds in its own run of factor entries),
// broadcasts the value with a lane read, shifts that lane's far sum into its
// near one, and every lane applies the step to both its sums with one FMA
// each.  The factor entries come from the zero-padded row and column forms
// as two contiguous 64-entry runs, with no bounds tests, and those for the
// next MG_INV_PD steps are in flight.  y and x live in LDS (x overwrites y);
// rows c .. n-1 of the column are written to row c of scr.
constexpr int MG_INV_WAVES = 2;

// Wait for this wave's LDS operations only (lgkmcnt = 0; vmcnt and expcnt
// left at their maxima), so prefetched global loads stay in flight.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

__global__ __launch_bounds__(64 * MG_INV_WAVES) void k_mg_coarse_inv(const MgChunk* __restrict__ chunks,
                                                                     const double* __restrict__ band,
                                                                     double* __restrict__ scr, int nmax) {
  extern __shared__ double ys_all[];  // [MG_INV_WAVES][nmax]
  constexpr int PD = MG_INV_PD;
  const MgChunk ch = chunks[blockIdx.y];
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * MG_INV_WAVES + wave);  // wave-uniform
  if (c >= n) return;  // whole wave
  const double* __restrict__ Lr = band + ch.band_off + PD * MG_BAND_RS;
  const double* __restrict__ Lc = band + ch.band_off + (int64_t)(n + 2 * PD) * MG_BAND_RS;
  double* ys = ys_all + wave * nmax;
  for (int i = lane; i < n; i += 64) ys[i] = 0.0;
  wait_lds();
  __builtin_amdgcn_wave_barrier();
  double pla[PD], plb[PD];
  // forward: near = the lane's smallest row >= i, far = near + 64; step i updates
  // rows i + 1 + t and i + 65 + t, t = (lane - i - 1) & 63 (column i of L); the
  // owner lane (t = 63) finds 1 / L[i][i] in its second entry
  auto fwd_load = [&](int i, double& la, double& lb) {
    const double* __restrict__ col = Lc + (int64_t)i * MG_BAND_CS;
    const int t = (lane - i - 1) & 63;
    la = col[t];
    lb = col[t + 64];
  };
  double an = lane == (c & 63) ? 1.0 : 0.0, af = 0.0;
#pragma unroll
  for (int d = 0; d < PD; ++d) fwd_load(c + d, pla[d], plb[d]);
  auto fwd_step = [&](int i, int d) {
    const int oi = i & 63;
    const double y = readlane_f64(an * plb[d], oi);
    const bool own = lane == oi;
    if (own) ys[i] = y;
    an = fma(-pla[d], y, own ? af : an);
    af = own ? 0.0 : fma(-plb[d], y, af);
    fwd_load(i + PD, pla[d], plb[d]);
  };
  int i0 = c;
  for (; i0 + PD <= n; i0 += PD) {  // full groups: no exits inside
#pragma unroll
    for (int d = 0; d < PD; ++d) fwd_step(i0 + d, d);
  }
#pragma unroll
  for (int d = 0; d < PD; ++d)
    if (i0 + d < n) fwd_step(i0 + d, d);  // uniform
  wait_lds();  // ys complete (each wave reads only its own ys; no block barrier, waves may have left)
  __builtin_amdgcn_wave_barrier();
  // backward: near = the lane's largest row <= i, far = near - 64; step i updates
  // rows i - 1 - u and i - 65 - u, u = (i - 1 - lane) & 63 (row i of L); sums
  // start at y; the owner lane (u = 63) finds 1 / L[i][i] in its second entry
  auto bwd_load = [&](int i, double& la, double& lb) {
    const double* __restrict__ row = Lr + (int64_t)i * MG_BAND_RS;
    const int u = (i - 1 - lane) & 63;
    la = row[1 + u];
    lb = row[65 + u];
  };
  {
    const int jn = n - 1 - ((n - 1 - lane) & 63);
    an = jn >= 0 ? ys[jn] : 0.0;
    af = jn >= 64 ? ys[jn - 64] : 0.0;
  }
#pragma unroll
  for (int d = 0; d < PD; ++d) bwd_load(n - 1 - d, pla[d], plb[d]);
  auto bwd_step = [&](int i, int d) {
    const int oi = i & 63;
    const double x = readlane_f64(an * plb[d], oi);
    const bool own = lane == oi;
    if (own) ys[i] = x;
    const double enter = i >= 128 ? ys[i - 128] : 0.0;  // the owner's new far row starts at y
    an = fma(-pla[d], x, own ? af : an);
    af = own ? enter : fma(-plb[d], x, af);
    bwd_load(i - PD, pla[d], plb[d]);
  };
  i0 = n - 1;
  for (; i0 - PD + 1 >= c; i0 -= PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) bwd_step(i0 - d, d);
  }
#pragma unroll
  for (int d = 0; d < PD; ++d)
    if (i0 - d >= c) bwd_step(i0 - d, d);  // uniform
  wait_lds();
  __builtin_amdgcn_wave_barrier();
  double* __restrict__ row = scr + ch.dense_off + (int64_t)c * n;
  for (int i = c + lane; i < n; i += 64) row[i] = ys[i];
}

// dense = P X P^T in natural order from the lower triangle of X (band
// numbering, column j stored from entry j on as row j of scr); P is the
// renumbering.  X is symmetric, so the upper triangle is its mirror.
__global__ __launch_bounds__(256) void k_mg_coarse_sym(const MgChunk* __restrict__ chunks, const double* __restrict__ scr,
                                                       double* __restrict__ dense) {
  const MgChunk ch = chunks[blockIdx.y];
  const int n = 2 * (ch.node_end - ch.node_begin);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
  auto band_of = [&](int d) {
    const int nq = d >> 1, x = nq % (ch.nx + 1), y = nq / (ch.nx + 1);
    return 2 * (ch.ny <= ch.nx ? x * (ch.ny + 1) + y : y * (ch.nx + 1) + x) + (d & 1);
  };
  const int bi = band_of(i), bj = band_of(j);
  const int lo = min(bi, bj), hi = max(bi, bj);
  dense[ch.dense_off + idx] = scr[ch.dense_off + (int64_t)lo * n + hi];
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

// ---- per-node steps of levels >= 1 ----

// Going up: e~ = e + P~ e2_coarse, then one l1-Jacobi sweep
// e2 = e~ + D^-1 (r - A e~).  Lane `sub` (< 9) of a node's 16-lane group
// forms e~ at stencil neighbour sub and its block product; the group sums the
// products with shuffles and the centre lane (sub 4) writes the node.  The
// chunk serves the systems sys .. sys + nsys - 1 of its instance: the
// neighbour's parents, weights, mask and the operator block are read once and
// used for every running system, whose vectors lie a level's node count apart.
// (The body of k_mg_prolong_smooth; ex0, ex1 receive the centre's result of
// system l for the level-1 injection.)
template <typename F>
__device__ __forceinline__ void mg_prolong_smooth_node(const MgChunk& ch, const PcgDev& s, int n, int sub,
                                                       bool node_ok, const double* __restrict__ A,
                                                       const double* __restrict__ mask,
                                                       const double* __restrict__ dinv,
                                                       const double* __restrict__ r, const double* __restrict__ e,
                                                       double* __restrict__ e2, F&& centre) {
  const int nx = ch.nx, ny = ch.ny, cnx = ch.cnx;
  const int64_t NN = (int64_t)(nx + 1) * (ny + 1), CN = (int64_t)(cnx + 1) * (ch.cny + 1);
  bool have = false;
  int64_t jo = 0, jn = 0, cvi[2][2];
  double wv[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, m0 = 0.0, m1 = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (node_ok && sub < 9) {
    const int ix = n % (nx + 1), iy = n / (nx + 1);
    const int jx = ix + sub % 3 - 1, jy = iy + sub / 3 - 1;
    if (jx >= 0 && jx <= nx && jy >= 0 && jy <= ny) {
      have = true;
      jo = (int64_t)jy * (nx + 1) + jx;
      jn = ch.op + jo;
      int px0, px1, py0, py1;
      double vx0, vx1, vy0, vy1;
      parents1d(jx, nx, px0, vx0, px1, vx1);
      parents1d(jy, ny, py0, vy0, py1, vy1);
      // a missing second parent (index -1, weight 0) reads the first one and adds 0
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a2_ = 0; a2_ < 2; ++a2_) {
          const int py = b == 0 || py1 < 0 ? py0 : py1;
          const int px = a2_ == 0 || px1 < 0 ? px0 : px1;
          cvi[b][a2_] = (int64_t)py * (cnx + 1) + px;
          const int pyw = b == 0 ? py0 : py1, pxw = a2_ == 0 ? px0 : px1;
          wv[b][a2_] = (pyw >= 0 && pxw >= 0) ? (a2_ == 0 ? vx0 : vx1) * (b == 0 ? vy0 : vy1) : 0.0;
        }
      m0 = mask[jn * 2];
      m1 = mask[jn * 2 + 1];
      const double* a = A + (ch.op + n) * 36 + sub * 4;
      a0 = a[0];
      a1 = a[1];
      a2 = a[2];
      a3 = a[3];
    }
  }
  for (int l = 0; l < ch.nsys; ++l) {
    if (!sys_running(s, ch.sys + l)) continue;  // uniform over the block
    const int64_t cvec = ch.cvec + l * CN, vec = ch.vec + l * NN;
    double et0 = 0.0, et1 = 0.0, c0 = 0.0, c1 = 0.0;
    if (have) {
      double c2[2][2][2];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a2_ = 0; a2_ < 2; ++a2_) {
          const int64_t cv = cvec + cvi[b][a2_];
          c2[b][a2_][0] = e2[cv * 2];
          c2[b][a2_][1] = e2[cv * 2 + 1];
        }
      double p0 = 0.0, p1 = 0.0;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a2_ = 0; a2_ < 2; ++a2_) {
          p0 += wv[b][a2_] * c2[b][a2_][0];
          p1 += wv[b][a2_] * c2[b][a2_][1];
        }
      const int64_t jv = vec + jo;
      et0 = e[jv * 2] + m0 * p0;
      et1 = e[jv * 2 + 1] + m1 * p1;
      c0 = a0 * et0 + a1 * et1;
      c1 = a2 * et0 + a3 * et1;
    }
    for (int o = 8; o > 0; o >>= 1) {
      c0 += __shfl_xor(c0, o, 16);
      c1 += __shfl_xor(c1, o, 16);
    }
    if (node_ok && sub == 4) {
      const int64_t node = ch.op + n, v = vec + n;
      const double out0 = et0 + dinv[node * 2] * (r[v * 2] - c0);
      const double out1 = et1 + dinv[node * 2 + 1] * (r[v * 2 + 1] - c1);
      e2[v * 2] = out0;
      e2[v * 2 + 1] = out1;
      centre(l, out0, out1);
    }
  }
}

// Levels l-1 -> l in one launch: r_l = R^T (mask * (r_{l-1} - A_{l-1} e_{l-1}))
// with the level l-1 residual formed where the restriction needs it.  16
// lanes per coarse node: lane k < 9 takes the fine node at offset
// (k % 3 - 1, k / 3 - 1) from the node's fine position, its weight and its
// 9-point residual; the 16 lanes sum with a fixed butterfly; then
// e_l = D^-1 r_l (pre-smoothing from zero).  A fine node is evaluated by each
// coarse node it restricts to (2.25 times on average) instead of being
// written and read back by a separate residual pass.
constexpr int MG_RR_NODES = 16;  // coarse nodes per 256-thread block

__global__ __launch_bounds__(256) void k_mg_resid_restrict(const MgChunk* __restrict__ chunks, PcgDev s,
                                                           const double* __restrict__ A,
                                                           const double* __restrict__ mask,
                                                           const double* __restrict__ dinv, double* __restrict__ r,
                                                           double* __restrict__ e) {
  const MgChunk ch = chunks[blockIdx.x];
  {  // the chunk serves systems sys .. sys + nsys - 1 of its instance
    bool any = false;
    for (int l = 0; l < ch.nsys; ++l) any |= sys_running(s, ch.sys + l);
    if (!any) return;  // whole block
  }
  const int sub = threadIdx.x & 15;
  const int n = ch.node_begin + blockIdx.y * MG_RR_NODES + (threadIdx.x >> 4);
  const bool node_ok = n < ch.node_end;
  const int fnx = ch.fnx, fny = ch.fny;
  const int64_t NN = (int64_t)(ch.nx + 1) * (ch.ny + 1), FN = (int64_t)(fnx + 1) * (fny + 1);
  // this lane's fine node, its weight and operator row: read once for all systems
  bool have = false;
  int fx = 0, fy = 0;
  int64_t fo = 0;
  double w = 0.0, m0 = 0.0, m1 = 0.0, a[9][4];
  if (node_ok && sub < 9) {
    const int cx = n % (ch.nx + 1), cy = n / (ch.nx + 1);
    fx = fine_of(cx, fnx) + sub % 3 - 1;
    fy = fine_of(cy, fny) + sub / 3 - 1;
    if (fx >= 0 && fx <= fnx && fy >= 0 && fy <= fny) {
      w = weight1d(fx, fnx, cx) * weight1d(fy, fny, cy);
      have = w != 0.0;
    }
  }
  if (have) {
    fo = (int64_t)fy * (fnx + 1) + fx;
    const int64_t fnode = ch.fop + fo;
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[k][q] = A[fnode * 36 + k * 4 + q];
    m0 = mask[fnode * 2];
    m1 = mask[fnode * 2 + 1];
  }
  for (int l = 0; l < ch.nsys; ++l) {
    if (!sys_running(s, ch.sys + l)) continue;  // uniform over the block
    const int64_t fvec = ch.fvec + l * FN, vec = ch.vec + l * NN;
    double acc0 = 0.0, acc1 = 0.0;
    if (have) {
      const int64_t fv = fvec + fo;
      double t0 = r[fv * 2], t1 = r[fv * 2 + 1];
      // all nine neighbours' loads are issued together (a neighbour off the
      // grid reads a clamped one and counts as 0), then used in order
      double ej[9][2];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int jx = fx + k % 3 - 1, jy = fy + k / 3 - 1;
        const bool in = jx >= 0 && jx <= fnx && jy >= 0 && jy <= fny;
        const int64_t jv = fvec + (int64_t)min(max(jy, 0), fny) * (fnx + 1) + min(max(jx, 0), fnx);
        const double v0 = e[jv * 2], v1 = e[jv * 2 + 1];
        ej[k][0] = in ? v0 : 0.0;
        ej[k][1] = in ? v1 : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        t0 -= a[k][0] * ej[k][0] + a[k][1] * ej[k][1];
        t1 -= a[k][2] * ej[k][0] + a[k][3] * ej[k][1];
      }
      acc0 = w * m0 * t0;
      acc1 = w * m1 * t1;
    }
    for (int o = 8; o > 0; o >>= 1) {
      acc0 += __shfl_xor(acc0, o, 16);
      acc1 += __shfl_xor(acc1, o, 16);
    }
    if (node_ok && sub == 0) {
      const int64_t node = ch.op + n, v = vec + n;
      r[v * 2] = acc0;
      r[v * 2 + 1] = acc1;
      e[v * 2] = dinv[node * 2] * acc0;
      e[v * 2 + 1] = dinv[node * 2 + 1] * acc1;
    }
  }
}

// Coarsest level: e2 = X r with the dense inverse X (natural order), one
// wave per row, the lanes over contiguous stretches of the row.
__global__ __launch_bounds__(256) void k_mg_coarse_solve(const MgChunk* __restrict__ chunks, PcgDev s,
                                                         const double* __restrict__ dense,
                                                         const double* __restrict__ r, double* __restrict__ e2) {
  constexpr int NL = 4;  // systems per pass over a row of X
  const MgChunk ch = chunks[blockIdx.y];
  const int nn = ch.node_end - ch.node_begin, n = 2 * nn;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;  // whole wave
  const double* __restrict__ X = dense + ch.dense_off + (int64_t)i * n;
  // the row of X is read once for up to NL systems of the instance
  for (int l0 = 0; l0 < ch.nsys; l0 += NL) {
    bool run[NL];
    bool any = false;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      run[l] = l0 + l < ch.nsys && sys_running(s, ch.sys + l0 + l);
      any |= run[l];
    }
    if (!any) continue;  // whole wave
    // eight terms per lane are requested before any is added (an eighth of
    // the memory round trips); each lane adds its terms in index order, an
    // absent one as 0 * 0, so each sum is the same as term by term
    double acc[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) acc[l] = 0.0;
    for (int j = lane; j < n; j += 512) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {  // unconditional (clamped) loads, absent terms zeroed after
        const int jj = min(j + 64 * u, n - 1);
        const double a0 = X[jj];
        x[u] = j + 64 * u < n ? a0 : 0.0;
      }
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        if (!run[l]) continue;
        const double* __restrict__ rv = r + (ch.vec + (int64_t)(l0 + l) * nn) * 2;
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int jj = min(j + 64 * u, n - 1);
          const double a1 = rv[jj];
          y[u] = j + 64 * u < n ? a1 : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[l] = fma(x[u], y[u], acc[l]);
      }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if (!run[l]) continue;
      double v = acc[l];
      for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
      if (lane == 0) e2[(ch.vec + (int64_t)(l0 + l) * nn) * 2 + i] = v;
    }
  }
}

// vfree != NULL (level 1): also z += e2 at the node's free vertex DOFs
// (the injection back to the hierarchic level), and the same correction into
// q at those DOFs (q is free between k_dof2 and the next k_dof1), from which
// the vertex-column product updates the slots.  MG_RR_NODES nodes per
// 256-thread block, 16 lanes each.
__global__ __launch_bounds__(256) void k_mg_prolong_smooth(const MgChunk* __restrict__ chunks, PcgDev s,
                                                           const double* __restrict__ A,
                                                           const double* __restrict__ mask,
                                                           const double* __restrict__ dinv,
                                                           const double* __restrict__ r, const double* __restrict__ e,
                                                           double* __restrict__ e2, const int32_t* __restrict__ vfree) {
  const MgChunk ch = chunks[blockIdx.x];
  {  // the chunk serves systems sys .. sys + nsys - 1 of its instance
    bool any = false;
    for (int l = 0; l < ch.nsys; ++l) any |= sys_running(s, ch.sys + l);
    if (!any) return;  // whole block
  }
  const int sub = threadIdx.x & 15;
  const int n = ch.node_begin + blockIdx.y * MG_RR_NODES + (threadIdx.x >> 4);
  const bool node_ok = n < ch.node_end;
  int f0 = -1, f1 = -1;
  if (vfree && node_ok && sub == 4) {
    const int64_t node = ch.op + n;
    f0 = vfree[node * 2];
    f1 = vfree[node * 2 + 1];
  }
  mg_prolong_smooth_node(ch, s, n, sub, node_ok, A, mask, dinv, r, e, e2, [&](int l, double o0, double o1) {
    if (!vfree) return;
    const int64_t dof = s.sys[ch.sys + l].dof_off;
    if (f0 >= 0) {
      s.z[dof + f0] += o0;
      s.q[dof + f0] = o0;
    }
    if (f1 >= 0) {
      s.z[dof + f1] += o1;
      s.q[dof + f1] = o1;
    }
  });
}

// Level 1 -> 0: z += injection^T e2_1 at the free vertex DOFs (and into q, as
// in k_mg_prolong_smooth).
__global__ __launch_bounds__(MGB) void k_mg_prolong0(const MgChunk* __restrict__ chunks, PcgDev s,
                                                     const int32_t* __restrict__ vfree, const double* __restrict__ e2) {
  const MgChunk ch = chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int n = ch.node_begin + threadIdx.x;
  if (n >= ch.node_end) return;
  const int64_t node = ch.op + n, v = ch.vec + n;
  for (int c = 0; c < 2; ++c) {
    const int f = vfree[node * 2 + c];
    if (f >= 0) {
      s.z[ch.dof_off + f] += e2[v * 2 + c];
      s.q[ch.dof_off + f] = e2[v * 2 + c];
    }
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
// threads of k_asm_block: fewer for the small blocks of p <= 2, so more
// elements are in flight per CU
template <int P>
constexpr int asm_block_threads() { return P == 1 ? 64 : P == 2 ? 128 : 256; }

// Position of (a, b), a <= b, in the row-packed upper triangle of an NE x NE matrix.
template <int NE>
__device__ __forceinline__ int packed_index(int a, int b) {
  return a * NE - (a * (a - 1)) / 2 + (b - a);
}
}

template <int P>
__global__ __launch_bounds__(asm_block_threads<P>()) void k_asm_block(const GroupDev* __restrict__ groups, int gi,
                                                         const int32_t* __restrict__ nbr,
                                                         const int32_t* __restrict__ el_group,
                                                         const int32_t* __restrict__ el_col,
                                                         const double* __restrict__ E, double* __restrict__ binv) {
  constexpr int NE = ne_of(P), ASM_BLOCK = asm_block_threads<P>();
  constexpr int NEMAX = ne_of(MTO_MAX_P);
  __shared__ double A[NE][NE + 1];
  __shared__ int gid[NE];
  __shared__ int posn[8][NEMAX];                       // each neighbour's DOFs in this element, or -1
  __shared__ double Esn[8][MTO_MAX_D * MTO_MAX_D];     // each neighbour's cell moduli
  __shared__ double Es[MTO_MAX_D * MTO_MAX_D];  // moduli of the element's cells
  // each neighbour's group data, fetched once (nb_p = -1: no neighbour)
  __shared__ int nb_p[8], nb_S[8], nb_npad[8], nb_cell[8], nb_cnt[8];
  __shared__ const int32_t* nb_gidx[8];  // the neighbour's column of its group's DOF table
  __shared__ const double* nb_ks[8];
  // Two elements share the DOFs of a common edge (at most 2 (P + 1) under the
  // minimum rule) or of a common vertex (2): four edge and four corner
  // neighbours give at most PAIRMAX shared DOF pairs.
  constexpr int SHMAX = 2 * (P + 1);
  constexpr int PAIRMAX = 4 * SHMAX * SHMAX + 4 * 4;
  __shared__ uint8_t nb_sh[8][SHMAX];  // the neighbour's local DOFs shared with this element
  __shared__ double nb_v[PAIRMAX];  // their entries, neighbour by neighbour
  const GroupDev g = groups[gi];
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < 8) {
    const int ge = nbr[tid * g.npad + k];
    int pn = -1;
    if (ge >= 0) {
      const GroupDev& gn = groups[el_group[ge]];
      const int kn = el_col[ge];
      pn = gn.p;
      nb_S[tid] = gn.S;
      nb_npad[tid] = gn.npad;
      nb_cell[tid] = gn.cell[kn];
      nb_gidx[tid] = gn.gidx + kn;
      nb_ks[tid] = gn.ks;
    }
    nb_p[tid] = pn;
  }
  for (int a = tid; a < NE; a += ASM_BLOCK) gid[a] = g.gidx[a * g.npad + k];
  const int cell = g.cell[k];
  for (int c = tid; c < g.S; c += ASM_BLOCK) Es[c] = E[cell + c];
  __syncthreads();
  // K_e = sum over cells of E_s K_s, the cell loop unrolled so that its
  // table loads are in flight together.  p >= 3: one thread per entry of the
  // upper triangle (packed order), mirrored (the K_s are symmetric, so both
  // triangles are the same sums); p <= 2: every entry (measured faster there).
  if constexpr (NE > 18) {
    constexpr int NT = NE * (NE + 1) / 2;
    for (int q = tid; q < NT; q += ASM_BLOCK) {
      // row a of packed entry q: rows start at a NE - a (a - 1) / 2
      int a = (int)((2 * NE + 1 - sqrtf((float)((2 * NE + 1) * (2 * NE + 1) - 8 * q))) * 0.5f);
      a = max(0, min(a, NE - 1));
      while (a > 0 && a * NE - a * (a - 1) / 2 > q) --a;
      while (a + 1 < NE && (a + 1) * NE - (a + 1) * a / 2 <= q) ++a;
      const int b = a + q - (a * NE - a * (a - 1) / 2);
      const double* __restrict__ kab = g.ks + (int64_t)a * NE + b;
      double v = 0.0;
#pragma unroll 8
      for (int sc_ = 0; sc_ < g.S; ++sc_) v = fma(Es[sc_], kab[(int64_t)sc_ * NE * NE], v);
      A[a][b] = v;
      A[b][a] = v;
    }
  } else {
    for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
      const int a = idx / NE, b = idx - a * NE;
      const double* __restrict__ kab = g.ks + (int64_t)a * NE + b;
      double v = 0.0;
#pragma unroll 4
      for (int sc_ = 0; sc_ < g.S; ++sc_) v = fma(Es[sc_], kab[(int64_t)sc_ * NE * NE], v);
      A[a][b] = v;
    }
  }
  __syncthreads();
  // neighbours: add their entries on pairs of shared DOFs (matched by free
  // index).  The DOF positions and cell moduli of all eight neighbours are
  // fetched in one phase, each neighbour's shared DOFs compacted with a wave
  // ballot, and the entries of every shared pair computed in one more phase;
  // the additions then run neighbour by neighbour, in order.
  for (int t2 = tid; t2 < 8 * NEMAX; t2 += ASM_BLOCK) {
    const int m = t2 / NEMAX, b = t2 - m * NEMAX;
    const int pn = nb_p[m];
    int ps = -1;
    if (pn >= 0 && b < ne_of(pn)) {
      const int id = nb_gidx[m][b * nb_npad[m]];
      if (id >= 0)
        for (int a = 0; a < NE; ++a)
          if (gid[a] == id) {
            ps = a;
            break;
          }
    }
    posn[m][b] = ps;
  }
  for (int t2 = tid; t2 < 8 * MTO_MAX_D * MTO_MAX_D; t2 += ASM_BLOCK) {
    const int m = t2 / (MTO_MAX_D * MTO_MAX_D), c = t2 - m * (MTO_MAX_D * MTO_MAX_D);
    if (nb_p[m] >= 0 && c < nb_S[m]) Esn[m][c] = E[nb_cell[m] + c];
  }
  __syncthreads();
  {
    const int wave = tid >> 6, lane = tid & 63;
    for (int m = wave; m < 8; m += ASM_BLOCK / 64) {
      const bool shared = lane < NEMAX && posn[m][lane] >= 0;
      const unsigned long long bal = __ballot(shared);
      const int pos = __popcll(bal & ((1ull << lane) - 1ull));
      if (shared && pos < SHMAX) nb_sh[m][pos] = (uint8_t)lane;
      if (lane == 0) nb_cnt[m] = min(__popcll(bal), SHMAX);
    }
  }
  __syncthreads();
  for (int t0 = tid; t0 < PAIRMAX; t0 += ASM_BLOCK) {
    int rem = t0, m = 0;
    for (; m < 8; ++m) {
      const int c = nb_cnt[m];
      if (rem < c * c) break;
      rem -= c * c;
    }
    if (m == 8) break;  // past the last pair
    const int c = nb_cnt[m], x = rem / c, y = rem - x * c;
    const int a = nb_sh[m][x], b = nb_sh[m][y], nen = ne_of(nb_p[m]);
    const double* __restrict__ kab = nb_ks[m] + (int64_t)a * nen + b;
    double v = 0.0;
#pragma unroll 8
    for (int sc_ = 0; sc_ < nb_S[m]; ++sc_) v = fma(Esn[m][sc_], kab[(int64_t)sc_ * nen * nen], v);
    nb_v[t0] = v;
  }
  __syncthreads();
  for (int m = 0, off = 0; m < 8; ++m) {  // uniform
    const int c = nb_cnt[m];
    if (c == 0) continue;
    for (int t = tid; t < c * c && off + t < PAIRMAX; t += ASM_BLOCK) {
      const int x = t / c, y = t - x * c;
      A[posn[m][nb_sh[m][x]]][posn[m][nb_sh[m][y]]] += nb_v[off + t];  // one-to-one within a neighbour
    }
    off += c * c;
    __syncthreads();
  }
  // absent or supported DOFs, and DOFs with no stiffness at all (E_min = 0
  // around them): marked by a diagonal of -1 and a zero row and column
  for (int a = tid; a < NE; a += ASM_BLOCK)
    if (!(A[a][a] > 0.0)) gid[a] = -1;
  __syncthreads();
  // upper triangle, packed by rows (the assembled block is symmetric: both
  // triangles are the same sums in the same order)
  for (int idx = tid; idx < NE * NE; idx += ASM_BLOCK) {
    const int a = idx / NE, b = idx - a * NE;
    if (b < a) continue;
    const double v = (gid[a] < 0 || gid[b] < 0) ? (a == b ? -1.0 : 0.0) : A[a][b];
    binv[(int64_t)k * asm_ntp_of(P) + packed_index<NE>(a, b)] = v;
  }
}

// In-place inverse of the element blocks by blocked Gauss-Jordan elimination
// on the matrix cores, one wave per element column: binv holds on entry the
// packed upper triangle written by k_asm_block (a marked DOF: diagonal -1,
// zero row) and on exit that of omega-free B_e, zero at marked DOFs.
//   The block, symmetrically scaled to unit diagonal (marked and padding DOFs:
//   identity rows), sits in MB x MB accumulator tiles of
//   v_mfma_f64_16x16x4f64 (tile (bi, bj), register r: row 16 bi + l/16 + 4 r,
//   column 16 bj + l%16 in lane l).  Step kb eliminates pivot rows
//   4 kb .. 4 kb + 3 (no pivoting: the block is SPD).  Their row panel Rr
//   is register r = kb % 4 of tile row kb / 4, in the B-operand layout as
//   it stands; the pivot block P is gathered from it with lane shuffles and
//   inverted in every lane.  Gauss-Jordan keeps the matrix symmetric between
//   rows and columns of the same kind (both eliminated or both not) and
//   antisymmetric between the kinds, so the column panel C in the A-operand
//   layout is Rr of the same lane with the sign of the eliminated rows
//   flipped.  Then, all on MFMA: R = P^-1 Rr, the rank-4 update A -= C R of
//   every tile, the new pivot columns -C P^-1; the pivot rows become R and
//   the pivot block P^-1.
template <int P>
__global__ __launch_bounds__(64, 2) void k_asm_invert(double* __restrict__ binv) {
  constexpr int NE = ne_of(P), NTP = asm_ntp_of(P), MB = mb_of(P), NB = (NE + 3) / 4;
  __shared__ double dg[16 * MB];
  const int lane = threadIdx.x, lr = lane >> 4, lc = lane & 15;
  double* __restrict__ bp = binv + (int64_t)blockIdx.x * NTP;
  auto pk = [](int a, int b) { return a <= b ? packed_index<NE>(a, b) : packed_index<NE>(b, a); };
  d4m acc[MB][MB];
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int bj = 0; bj < MB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * bi + lr + 4 * r, b = 16 * bj + lc;
        acc[bi][bj][r] = (a < NE && b < NE) ? bp[pk(a, b)] : (a == b ? 1.0 : 0.0);
      }
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (lc == lr + 4 * r) dg[16 * bi + lc] = acc[bi][bi][r];
  __syncthreads();
  // symmetric scaling to unit diagonal (factor 0 at marked DOFs, whose
  // rows become identity rows); the factors are kept in LDS for the end
  __syncthreads();
  if (lane < 16 * MB) dg[lane] = dg[lane] > 0.0 ? 1.0 / sqrt(dg[lane]) : 0.0;
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int bj = 0; bj < MB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * bi + lr + 4 * r, b = 16 * bj + lc;
        const double sa = dg[a];
        const double v = acc[bi][bj][r] * sa * dg[b];
        acc[bi][bj][r] = (a == b && !(sa > 0.0)) ? 1.0 : v;
      }
  const d4m zero = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kb = 0; kb < NB; ++kb) {
    const int bk = kb / 4, rk = kb % 4, pc0 = 4 * (kb % 4);
    double Rr[MB];
#pragma unroll
    for (int bj = 0; bj < MB; ++bj) Rr[bj] = acc[bk][bj][rk];
    // the pivot block, then its inverse (Gauss-Jordan on 4 x 4, every lane)
    double M[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) M[q][c] = __shfl(Rr[bk], 16 * q + pc0 + c);
#pragma unroll
    for (int t0 = 0; t0 < 4; ++t0) {
      const double ip = 1.0 / M[t0][t0];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j != t0) M[t0][j] *= ip;
      M[t0][t0] = ip;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i == t0) continue;
        const double f = M[i][t0];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j != t0) M[i][j] -= f * M[t0][j];
        M[i][t0] = -f * ip;
      }
    }
    // P^-1 as an A operand (rows 0..3) and as a B operand at the pivot columns
    double piA = 0.0, piB = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (lc == q && lr == c) piA = M[q][c];
        if (lr == q && lc == pc0 + c) piB = M[q][c];
      }
    const bool pcol = lc >= pc0 && lc < pc0 + 4;
    double RB[MB], CA[MB];
#pragma unroll
    for (int bj = 0; bj < MB; ++bj) {
      const d4m t = __builtin_amdgcn_mfma_f64_16x16x4f64(piA, Rr[bj], zero, 0, 0, 0);
      RB[bj] = t[0];  // R = P^-1 Rr: lane l holds R[l/16][16 bj + l%16]
      CA[bj] = (16 * bj + lc < 4 * kb) ? Rr[bj] : -Rr[bj];  // -C, eliminated rows sign-flipped
    }
    // the new pivot columns -C P^-1 first; the update below then leaves them
    // alone (R is taken as zero there)
#pragma unroll
    for (int bi = 0; bi < MB; ++bi) {
      const d4m x = __builtin_amdgcn_mfma_f64_16x16x4f64(CA[bi], piB, zero, 0, 0, 0);
      if (pcol) acc[bi][bk] = x;
    }
    const double rbk = RB[bk];
    if (pcol) RB[bk] = 0.0;
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(CA[bi], RB[bj], acc[bi][bj], 0, 0, 0);
    // the pivot rows become R, the pivot block P^-1
    RB[bk] = pcol ? piB : rbk;
#pragma unroll
    for (int bj = 0; bj < MB; ++bj) acc[bk][bj][rk] = RB[bj];
  }
  // unscale; upper triangle, packed by rows
#pragma unroll
  for (int bi = 0; bi < MB; ++bi)
#pragma unroll
    for (int bj = bi; bj < MB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * bi + lr + 4 * r, b = 16 * bj + lc;
        if (a <= b && b < NE) bp[packed_index<NE>(a, b)] = acc[bi][bj][r] * dg[a] * dg[b];
      }
}

// slots2 = omega * B_e v_e.  A persistent grid (as many blocks of 256
// threads as fit on the chip at once) walks the tiles of EB = asm_cols_of(P)
// element columns of each instance's first system; block b takes the tiles
// b, b + G, b + 2G, ... (G blocks) whose instance still has a running system,
// found by all its threads at once and listed in LDS.  Thread (column c,
// row a) serves the first NE EB threads.  A tile's packed triangles are one
// contiguous range of binv, read with 16-byte loads by all threads and staged
// in LDS, where each entry serves rows a and b; row a then sums B(a, b) v_b in
// order of b.  The loads are software-pipelined: while a tile is computed
// from LDS, the next tile's triangles and element vectors and the tile after
// it's gather indices are in flight in registers, so HBM stays busy through
// the LDS-bound sums.  Up to ASM_SYS systems of the instance per pass: the
// element blocks are shared by its load cases, so one read of a block serves
// all of them (an instance with more systems takes further passes, whose
// element vectors are gathered in place).
constexpr int ASM_SYS = 4;
constexpr int ASM_THREADS = 256;
constexpr int ASM_PERSIST_MIN = 4;

template <int P>
__global__ __launch_bounds__(ASM_THREADS, 3) void k_asm_apply(GroupDev g, const Tile* __restrict__ tiles,
                                                           const double* __restrict__ binv,
                                                           const double* __restrict__ v, PcgDev s,
                                                           double* __restrict__ out_slots, double omega, int resid) {
  constexpr int NE = ne_of(P), NTP = asm_ntp_of(P), EB = asm_cols_of(P);
  static_assert(NE * EB <= ASM_THREADS, "one thread per row and column");
  constexpr int NB2 = EB * NTP / 2;                          // 16-byte words of a tile's triangles
  constexpr int LPT = (NB2 + ASM_THREADS - 1) / ASM_THREADS;  // of those, per thread
  constexpr int NW = ASM_THREADS / 64;
  __shared__ double2 bs2[NB2];
  __shared__ double vs[ASM_SYS][EB][NE];
  __shared__ int list[ASM_THREADS];
  __shared__ int wcount[NW];
  const double* bs = (const double*)bs2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid / NE, a = tid - c * NE;
  const int64_t n = g.ms_n_tiles;
  const Tile* __restrict__ tl = tiles + g.ms_tile_begin;  // nsys of the tile's instance in pc_begin

  auto running = [&](const Tile& t) {
    bool any = false;
    for (int l = 0; l < t.pc_begin; ++l) any |= s.status[t.sys + l] == SYS_RUNNING;
    return any;
  };
  // gather indices of this thread's row of a tile (-1: no row, or a supported DOF)
  auto indices = [&](const Tile& t, int& id, int& si) {
    id = si = -1;
    if (c < EB && c < t.count) {  // thread tid of the tile's contiguous run
      const int2 q = ((const int2*)g.msidx)[(int64_t)t.elem_begin * NE + tid];
      id = q.x;
      si = q.y;
    }
  };
  // a tile's triangles (words of absent columns of a partial last tile are not read)
  auto triangles = [&](const Tile& t, double2 (&stg)[LPT]) {
    const double2* __restrict__ src = (const double2*)(binv + (int64_t)t.elem_begin * NTP);
    const int nw = t.count * (NTP / 2);
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int i = tid + ASM_THREADS * k;
      stg[k] = i < nw ? src[i] : double2{0.0, 0.0};
    }
  };
  // element-vector entries of systems l0 .. l0 + ASM_SYS - 1 of a tile's
  // instance (zero for a stopped system or no DOF); bit l of run: system l0 + l runs
  auto gather = [&](const Tile& t, int l0, int id, double (&x)[ASM_SYS], unsigned& run) {
    const int np = min(ASM_SYS, t.pc_begin - l0);
    run = 0;
#pragma unroll
    for (int l = 0; l < ASM_SYS; ++l) {
      x[l] = 0.0;
      if (l >= np) continue;
      const int sys = t.sys + l0 + l;
      if (s.status[sys] != SYS_RUNNING) continue;  // the same address in every lane: one load
      run |= 1u << l;
      if (id >= 0) {
        const SysDesc& sd = s.sys[sys];
        const double* __restrict__ vsys = v + sd.dof_off;
        x[l] = resid ? vsys[id] - slot_sum(s.slots + sd.slot_off, id, sd.nfv, sd.nfe) : vsys[id];
      }
    }
  };
  // rows of one pass from LDS; slots2 of the running systems
  const int ra = a * NE - (a * (a - 1)) / 2 - a;  // row a: entry (min, max) at cb + a (b < a) or ra + b
  auto rows = [&](const Tile& t, int l0, int si, unsigned run) {
    const int np = min(ASM_SYS, t.pc_begin - l0);
    if (!(c < EB && c < t.count)) return;
    const double* __restrict__ brow = bs + c * NTP;
    double acc[ASM_SYS] = {0.0, 0.0, 0.0, 0.0};
    const double* __restrict__ vc = &vs[0][c][0];
    auto sum = [&](auto nl) {
      constexpr int NL = decltype(nl)::value;
#pragma unroll 5
      for (int b = 0; b < NE; ++b) {
        const int cb = b * NE - (b * (b - 1)) / 2 - b;
        const double e = brow[b < a ? cb + a : ra + b];
#pragma unroll
        for (int l = 0; l < NL; ++l) acc[l] = fma(e, vc[l * EB * NE + b], acc[l]);
      }
    };
    switch (np) {  // uniform over the block
      case 1: sum(std::integral_constant<int, 1>{}); break;
      case 2: sum(std::integral_constant<int, 2>{}); break;
      case 3: sum(std::integral_constant<int, 3>{}); break;
      default: sum(std::integral_constant<int, 4>{}); break;
    }
    if (si < 0) return;
#pragma unroll
    for (int l = 0; l < ASM_SYS; ++l)
      if ((run >> l) & 1u) out_slots[s.sys[t.sys + l0 + l].slot_off + si] = omega * acc[l];
  };
  auto put_vectors = [&](const Tile& t, const double (&x)[ASM_SYS]) {
    if (!(c < EB)) return;
#pragma unroll
    for (int l = 0; l < ASM_SYS; ++l) vs[l][c][a] = x[l];
  };

  // tiles at(0), ..., at(cnt - 1) (uniform tile indices): tile i is summed
  // from LDS while tile i + 1's data and tile i + 2's indices load
  auto pipeline = [&](int cnt, auto at) {
    Tile tn = tl[at(0)];
    double2 stg[LPT];
    int id, si, id2 = -1, si2 = -1;
    double x[ASM_SYS];
    unsigned run;
    triangles(tn, stg);
    indices(tn, id, si);
    Tile tn2 = tn;
    if (cnt > 1) {
      tn2 = tl[at(1)];
      indices(tn2, id2, si2);
    }
    gather(tn, 0, id, x, run);
    for (int i = 0; i < cnt; ++i) {
      const Tile t = tn;
      const int cur_id = id, cur_si = si;
      const unsigned cur_run = run;
      __syncthreads();  // the previous tile's sums have finished with bs2 and vs
#pragma unroll
      for (int k = 0; k < LPT; ++k) {
        const int j = tid + ASM_THREADS * k;
        if (j < NB2) bs2[j] = stg[k];
      }
      put_vectors(t, x);
      if (i + 1 < cnt) {
        tn = tn2;
        id = id2;
        si = si2;
        triangles(tn, stg);
        if (i + 2 < cnt) {
          tn2 = tl[at(i + 2)];
          indices(tn2, id2, si2);
        }
      }
      __syncthreads();  // the tile's triangles and element vectors are in LDS
      rows(t, 0, cur_si, cur_run);
      if (i + 1 < cnt) gather(tn, 0, id, x, run);
      for (int l0 = ASM_SYS; l0 < t.pc_begin; l0 += ASM_SYS) {  // instances with more systems
        double xx[ASM_SYS];
        unsigned rr;
        gather(t, l0, cur_id, xx, rr);
        __syncthreads();  // vs is free again
        put_vectors(t, xx);
        __syncthreads();
        rows(t, l0, cur_si, rr);
      }
    }
  };

  if (gridDim.x >= n) {  // one tile per block (small launches): no list
    if (blockIdx.x >= n) return;  // uniform over the block
    const int ti = xcd_tile(blockIdx.x, (int)n, g.xcd_run);
    if (!running(tl[ti])) return;
    pipeline(1, [&](int) { return ti; });
    return;
  }
  for (int64_t w0 = blockIdx.x; w0 < n; w0 += (int64_t)gridDim.x * ASM_THREADS) {
    // this block's tiles w0 + k G, k = 0 .. 255, that still have work: listed in order
    __syncthreads();  // list and wcount of the previous window are no longer read
    // candidate w0 + tid G runs on this block's XCD (G is a multiple of 8);
    // xcd_tile maps it to a tile so that each XCD takes neighbouring tiles
    const int64_t vi = w0 + (int64_t)tid * gridDim.x;
    const int ti = vi < n ? xcd_tile((int)vi, (int)n, g.xcd_run) : 0;
    const bool on = vi < n && running(tl[ti]);
    const uint64_t bal = __ballot(on);
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, cnt = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      off += w < wave ? wcount[w] : 0;
      cnt += wcount[w];
    }
    if (on) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = ti;
    __syncthreads();
    if (cnt == 0) continue;  // uniform over the block
    pipeline(cnt, [&](int i) { return __builtin_amdgcn_readfirstlane(list[i]); });
  }
}

// z = assembled slots2 (the Schwarz products)
__global__ __launch_bounds__(1024) void k_asm_z(PcgDev s, const double* __restrict__ slots2) {
  const Chunk ch = s.chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int i = ch.begin + threadIdx.x;
  if (i >= ch.end) return;
  s.z[ch.dof_off + i] = slot_sum(slots2 + ch.slot_off, i, ch.nfv, ch.nfe);
}

// z += assembled slots; partial sums of r.z for the next PCG iteration
__global__ __launch_bounds__(1024) void k_asm_post(PcgDev s, const double* __restrict__ slots2, int it_k, int init) {
  __shared__ double lds[20];
  const Chunk ch = s.chunks[blockIdx.x];
  if (!sys_running(s, ch.sys)) return;
  const int par = init ? 0 : ((*s.it_base + it_k + 1) & 1);
  const int i = ch.begin + threadIdx.x;
  double arz = 0.0;
  if (i < ch.end) {
    const int64_t o = ch.dof_off + i;
    const double zi = s.z[o] + slot_sum(slots2 + ch.slot_off, i, ch.nfv, ch.nfe);
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
void launch_mg_coarse_factor(const MgChunk* ch, int n, int bmax, const double* A, double* band, hipStream_t st) {
  if (!n) return;
  if (chol_panel_rows(bmax) <= 64)
    hipLaunchKernelGGL(k_mg_coarse_chol<1>, dim3(n), dim3(MG_CHOL_BLOCK), chol_lds_bytes(bmax), st, ch, A, band);
  else
    hipLaunchKernelGGL(k_mg_coarse_chol<2>, dim3(n), dim3(MG_CHOL_BLOCK), chol_lds_bytes(bmax), st, ch, A, band);
}
void launch_mg_coarse_inverse(const MgChunk* ch, int n, int nmax, double* band, double* scr, double* dense,
                              hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_mg_coarse_inv, dim3((nmax + MG_INV_WAVES - 1) / MG_INV_WAVES, n), dim3(64 * MG_INV_WAVES),
                     (size_t)MG_INV_WAVES * nmax * 8, st, ch, band, scr, nmax);
  const int64_t nn = (int64_t)nmax * nmax;
  hipLaunchKernelGGL(k_mg_coarse_sym, dim3((unsigned)((nn + 255) / 256), n), dim3(256), 0, st, ch, scr, dense);
}
void launch_mg_restrict0(const MgChunk* ch, int n, const PcgDev& s, const int32_t* vfree, const double* dinv,
                         double* r1, double* e1, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_restrict0, dim3(n), dim3(MGB), 0, st, ch, s, vfree, dinv, r1, e1);
}
void launch_mg_resid_restrict(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* mask,
                              const double* dinv, double* r, double* e, hipStream_t st) {
  if (n)
    hipLaunchKernelGGL(k_mg_resid_restrict, dim3(n, MG_CHUNK / MG_RR_NODES), dim3(256), 0, st, ch, s, A, mask, dinv,
                       r, e);
}
void launch_mg_coarse_solve(const MgChunk* ch, int n, int nmax, const PcgDev& s, const double* dense, const double* r,
                            double* e2, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_mg_coarse_solve, dim3((nmax + 3) / 4, n), dim3(256), 0, st, ch, s, dense, r, e2);
}
void launch_mg_prolong_smooth(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* mask,
                              const double* dinv, const double* r, const double* e, double* e2, const int32_t* vfree,
                              hipStream_t st) {
  if (n)
    hipLaunchKernelGGL(k_mg_prolong_smooth, dim3(n, MG_CHUNK / MG_RR_NODES), dim3(256), 0, st, ch, s, A, mask, dinv, r,
                       e, e2, vfree);
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
  const dim3 grid(g.n_elems);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_asm_block<1>, grid, dim3(asm_block_threads<1>()), 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
    case 2: hipLaunchKernelGGL(k_asm_block<2>, grid, dim3(asm_block_threads<2>()), 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
    case 3: hipLaunchKernelGGL(k_asm_block<3>, grid, dim3(asm_block_threads<3>()), 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
    default: hipLaunchKernelGGL(k_asm_block<4>, grid, dim3(asm_block_threads<4>()), 0, st, groups, gi, nbr, el_group, el_col, E, binv); break;
  }
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_asm_invert<1>, grid, dim3(64), 0, st, binv); break;
    case 2: hipLaunchKernelGGL(k_asm_invert<2>, grid, dim3(64), 0, st, binv); break;
    case 3: hipLaunchKernelGGL(k_asm_invert<3>, grid, dim3(64), 0, st, binv); break;
    default: hipLaunchKernelGGL(k_asm_invert<4>, grid, dim3(64), 0, st, binv); break;
  }
}
// Blocks of k_asm_apply<p> resident on the current device at once (cached per
// device and order).
static int asm_apply_blocks(int p) {
  static int cache[64][4];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int& nb = cache[dev][p - 1];
  if (nb > 0) return nb;
  int per_cu = 0, cus = 0;
  hipError_t e;
  switch (p) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_asm_apply<1>, ASM_THREADS, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_asm_apply<2>, ASM_THREADS, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_asm_apply<3>, ASM_THREADS, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_asm_apply<4>, ASM_THREADS, 0); break;
  }
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  nb = per_cu * cus;
  return nb;
}

void launch_asm_apply(const GroupDev& g, const Tile* tiles, const double* binv, const double* v, int resid,
                      const PcgDev& s, double* slots2, double omega, hipStream_t st) {
  if (g.ms_n_tiles == 0) return;
  // persistent: the blocks that fit on the device at once, at most one per
  // tile.  MTO_ASM_GRID (a positive integer) caps the count: the results do
  // not depend on it (every tile is summed the same way by whichever block
  // takes it), which lets tests run the pipeline and the tile windows of a
  // large grid on small meshes.
  // Launches of fewer than ASM_PERSIST_MIN tiles per resident block take one
  // block per tile instead (the walk's list costs more than it saves there).
  int nb = asm_apply_blocks(g.p);
  if (g.ms_n_tiles < ASM_PERSIST_MIN * nb) nb = g.ms_n_tiles;
  // a multiple of 8 blocks, so that block b and its candidates b + k G share XCD b mod 8
  nb = (std::min(g.ms_n_tiles, nb) + 7) / 8 * 8;
  if (const char* cap = std::getenv("MTO_ASM_GRID")) {
    const int c = std::atoi(cap);
    if (c > 0) nb = std::min(nb, c);
  }
  const dim3 grid(nb), block(ASM_THREADS);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_asm_apply<1>, grid, block, 0, st, g, tiles, binv, v, s, slots2, omega, resid); break;
    case 2: hipLaunchKernelGGL(k_asm_apply<2>, grid, block, 0, st, g, tiles, binv, v, s, slots2, omega, resid); break;
    case 3: hipLaunchKernelGGL(k_asm_apply<3>, grid, block, 0, st, g, tiles, binv, v, s, slots2, omega, resid); break;
    default: hipLaunchKernelGGL(k_asm_apply<4>, grid, block, 0, st, g, tiles, binv, v, s, slots2, omega, resid); break;
  }
}
void launch_asm_z(const PcgDev& s, const double* slots2, hipStream_t st) {
  hipLaunchKernelGGL(k_asm_z, dim3(s.n_chunks), dim3(1024), 0, st, s, slots2);
}
void launch_asm_post(const PcgDev& s, const double* slots2, int it_k, int init, hipStream_t st) {
  hipLaunchKernelGGL(k_asm_post, dim3(s.n_chunks), dim3(1024), 0, st, s, slots2, it_k, init);
}


}  // namespace mto
