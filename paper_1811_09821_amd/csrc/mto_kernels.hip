// HIP kernels (gfx950) of the FEA + sensitivity step: SIMP moduli, the
// element contraction on FP64 MFMA, the deterministic slot scatter and the
// fused PCG vector kernels, and the sensitivity contraction.
//
// Element contraction (the matvec of the PCG, K never assembled): for an
// element group with order p and a d x d cell grid, y_e = sum_s E_{e,s} K_s u_e
// (Sec. 2.2 stiffness with the composite integration of Appendix B).  Written
// as one GEMM per group, Y[n_e x cols] = Kcat[n_e x S*NEP] W[S*NEP x cols] with
// W[(s, j), e] = E_{e,s} u_e[j]: the shared table Kcat is the MFMA A operand and
// W is formed on the fly from gathered u_e (one multiply per MFMA B operand).
// v_mfma_f64_16x16x4f64 lane layout (checked on gfx950): A lane l holds
// A[l%16][l/16], B lane l holds B[l/16][l%16], D lane l holds D[l/16 + 4r][l%16].
//
// PCG (Jacobi preconditioner), per system (instance x load case), iteration i
// with parity pi = i & 1:
//   elem   p = z + beta p on the fly, element results to slots
//   dof1   q = sum of slots, p written, partial p.q
//   dof2   alpha = rz / pq, x += alpha p, r -= alpha q, z = D^-1 r, partial r.z, r.r
// Scalars are never stored: every kernel re-reduces the per-chunk partial sums
// of its system with one fixed wave-level order, so all blocks of all kernels
// see bit-identical alpha, beta and convergence decisions.

#include <hip/hip_runtime.h>

#include <type_traits>
#include <hip/hip_ext.h>

#include "mto_kernels.hpp"

namespace mto {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
// Vector kernels: one block per chunk of VBLOCK free DOFs of one system.
constexpr int VBLOCK = 1024;
constexpr int VWAVES = VBLOCK / 64;

// Sum of arr[a..b) by one wave: strided sequential sums per lane, then a xor
// butterfly.  Every lane ends with the same bits, and so does every wave that
// calls it on the same range.
__device__ __forceinline__ double wave_sum(const double* __restrict__ arr, int a, int b) {
  const int lane = threadIdx.x & 63;
  // four loads per lane are requested before any is added (a quarter of the
  // memory round trips); each lane still adds its terms in index order, an
  // absent term as +0.0, so the sum is the same as term by term
  double v = 0.0;
  for (int k = a + lane; k < b; k += 256) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // unconditional (clamped) loads, absent terms zeroed after
      const double t = arr[min(k + 64 * u, b - 1)];
      x[u] = k + 64 * u < b ? t : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) v += x[u];
  }
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// N wave_sum reductions over the same chunk range in one pass: each
// array's terms are added in wave_sum's order, so the results are identical
// to N calls, at one memory round trip instead of N.
template <int N>
__device__ __forceinline__ void wave_sum_n(const double* const (&arr)[N], int a, int b, double (&out)[N]) {
  const int lane = threadIdx.x & 63;
  double v[N];
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = 0.0;
  for (int k = a + lane; k < b; k += 256) {
    double tv[N][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // unconditional (clamped) loads, absent terms zeroed after
      const int kk = min(k + 64 * u, b - 1);
      const bool in = k + 64 * u < b;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const double x = arr[j][kk];
        tv[j][u] = in ? x : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < N; ++j) v[j] += tv[j][u];
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], m);
#pragma unroll
  for (int j = 0; j < N; ++j) out[j] = v[j];
}

// The stop threshold of a PCG cycle on r.r: rtol^2 f.f, or, when larger, the
// rounding floor of the cycle's residual recurrence, (4 eps ||D x||)^2 with
// D = diag(K) (xx = sum of (D x)_i^2 over the system).  Below that floor the
// recursive residual keeps falling but the true residual of x does not (the
// FP64 product K x carries errors of about eps |K| |x|, large where regions
// joined to the supports through void material move far); the cycle stops
// there and the refinement restart, from the double-double true residual,
// continues with a small correction.  4 eps ||D x|| is about the floor
// measured on the mixed batch (its true residual after the cycle is 2.6 to
// 3.9 times eps ||D x||), and far below rtol ||f|| where x stays moderate.
__device__ __forceinline__ double stop_thr2(const PcgDev& s, int sys, double xx) {
  constexpr double G2 = 16.0 * 0x1p-106;  // (4 eps)^2, eps = 2^-53
  return fmax(s.tol2[sys], G2 * xx);
}

template <int NW>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) t += lds[w];
  return t;
}

struct Scal {
  bool active;
  double beta;
};

// Convergence state and beta of system `sys` (partial sums in chunks
// [pc_begin, pc_end)) at iteration `it`.  A newly converged system is latched
// by a designated thread of the caller.
__device__ __forceinline__ Scal pcg_state(const PcgDev& s, int sys, int pc_begin, int pc_end, int it,
                                          bool want_beta) {
  const int pi = it & 1;
  const int st = s.status[sys];
  double rr, xx, rz_new = 0.0, rz_old = 1.0;
  if (want_beta && it > 0) {
    const double* const arr[4] = {s.part_rr + pi * s.n_chunks, s.part_rz + pi * s.n_chunks,
                                  s.part_rz + (pi ^ 1) * s.n_chunks, s.part_xx + pi * s.n_chunks};
    double out[4];
    wave_sum_n<4>(arr, pc_begin, pc_end, out);
    rr = out[0];
    rz_new = out[1];
    rz_old = out[2];
    xx = out[3];
  } else {
    const double* const arr[2] = {s.part_rr + pi * s.n_chunks, s.part_xx + pi * s.n_chunks};
    double out[2];
    wave_sum_n<2>(arr, pc_begin, pc_end, out);
    rr = out[0];
    xx = out[1];
  }
  Scal o;
  o.active = (st == SYS_RUNNING) && !(rr <= stop_thr2(s, sys, xx));
  o.beta = (want_beta && it > 0) ? rz_new / rz_old : 0.0;
  return o;
}

// ---------------------------------------------------------------------------
// Double-double arithmetic for the accurate residual f - K x (error-free
// transformations: Knuth's two-sum, FMA-based two-product).  Contraction of
// the rounded operations into FMAs is switched off inside these helpers.
struct dd_t {
  double hi, lo;
};

__device__ __forceinline__ dd_t two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd_t{s, e};
}

__device__ __forceinline__ dd_t dd_add(dd_t x, dd_t y) {
#pragma clang fp contract(off)
  const dd_t s = two_sum(x.hi, y.hi);
  const double lo = s.lo + (x.lo + y.lo);
  return two_sum(s.hi, lo);
}

// x + a * b for doubles a, b
__device__ __forceinline__ dd_t dd_fma(dd_t x, double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double e = fma(a, b, -p);
  return dd_add(x, dd_t{p, e});
}

// a * y for a double a
__device__ __forceinline__ dd_t dd_scale(double a, dd_t y) {
#pragma clang fp contract(off)
  const double p = a * y.hi;
  const double e = fma(a, y.hi, -p);
  const double lo = fma(a, y.lo, e);
  return two_sum(p, lo);
}

// Element contraction in extended precision: y_e = sum_s E_s (K_s x_e), each
// cell's row sum as a compensated dot product (as if in twice FP64's
// precision), scaled by E_s and summed over the cells in double-double;
// results to (slots, slots_lo).  Used only for the true residual.  One block per 16 element columns of a tile
// (blockIdx.y picks the part), one thread per (row, column); x_e (high and
// low parts) is gathered once into LDS.
// The rigid motion r_e through x_e's DOFs 0, 1 (vertex (0,0)) and 3 (vertex
// (1,0) y) is removed from x_e first: K_s r_e = 0 exactly, so the result is
// the same operator, but the FP64 tables annihilate rigid motions only to
// their rounding, and a region joined to the supports through void material
// moves rigidly by ~1e9 times its deformation; applied to that motion the
// tables' rounding would put spurious forces of ~1e-7 relative size into
// the residual.
template <int P>
constexpr int dd_rows() { return (ne_of(P) + 3) / 4 * 4; }

template <int P>
__global__ __launch_bounds__(16 * dd_rows<P>()) void k_elem_dd(GroupDev g, const Tile* __restrict__ tiles,
                                                             const double* __restrict__ E,
                                                             const double* __restrict__ xhi,
                                                             const double* __restrict__ xlo,
                                                             double* __restrict__ slots,
                                                             double* __restrict__ slots_lo,
                                                             const int32_t* __restrict__ skip) {
  constexpr int NE = ne_of(P);
  __shared__ double uh[NE][17], ul[NE][17];
  const Tile t = tiles[g.tile_begin + blockIdx.x];
  const int c0 = blockIdx.y * 16;
  // uniform over the block; skip[sys] != 0: not wanted (a system that did not
  // run since its last true residual still has it in the slots)
  if (c0 >= t.count || skip[t.sys]) return;
  const int c = threadIdx.x & 15, row = threadIdx.x >> 4;
  const bool valid = c0 + c < t.count;
  const int el = t.elem_begin + c0 + (valid ? c : 0);
  if (row < NE) {
    const int gi = valid ? g.gidx[row * g.npad + el] : -1;
    uh[row][c] = gi >= 0 ? xhi[t.dof_off + gi] : 0.0;
    ul[row][c] = gi >= 0 ? xlo[t.dof_off + gi] : 0.0;
  }
  __syncthreads();
  {
    // rigid motion (a - th y, b + th x): a = x_0, b = x_1, th = x_3 - x_1
    const dd_t a{uh[0][c], ul[0][c]}, b{uh[1][c], ul[1][c]};
    const dd_t th = dd_add(dd_t{uh[3][c], ul[3][c]}, dd_t{-b.hi, -b.lo});
    __syncthreads();
    if (row < 8) {  // vertex k = row / 2 at (i, j) = (k & 1, k >> 1), component row & 1
      const int k = row >> 1, i = k & 1, j = k >> 1, dof = 2 * (j * (P + 1) + i) + (row & 1);
      const dd_t r = (row & 1) ? (i ? dd_add(b, th) : b) : (j ? dd_add(a, dd_t{-th.hi, -th.lo}) : a);
      const dd_t v = dd_add(dd_t{uh[dof][c], ul[dof][c]}, dd_t{-r.hi, -r.lo});
      uh[dof][c] = v.hi;
      ul[dof][c] = v.lo;
    }
    __syncthreads();
  }
  if (row >= NE || !valid) return;
  const int si = g.sidx[row * g.npad + el];
  if (si < 0) return;
  const int cb = g.cell[el];
  dd_t y{0.0, 0.0};
  // Each cell's row sum is a compensated dot product (Ogita, Rump and Oishi's
  // Dot2): the running sum p carries the leading part, every product's
  // rounding error (from an FMA) and every addition's (TwoSum) go into one
  // FP64 correction s; p + s is then as accurate as a sum in twice the
  // working precision, rounded.  That bound (relative 2^-53 plus
  // (n 2^-53)^2 of the sum of |terms|) is far below the rtol of any test
  // while costing 11 FP64 operations per term.
  for (int sc = 0; sc < g.S; ++sc) {
    const double* __restrict__ kr = g.ks + ((size_t)sc * NE + row) * NE;
    double p = 0.0, s = 0.0;
#pragma unroll 10
    for (int j = 0; j < NE; ++j) {
      const double a = kr[j], b = uh[j][c];
      const double h = a * b;
      const double e = fma(a, b, -h);
      const dd_t ps = two_sum(p, h);
      p = ps.hi;
      s += ps.lo + e;
      s = fma(a, ul[j][c], s);  // low part of x: one rounding at ~2^-106 relative
    }
    y = dd_add(y, dd_scale(E[cb + sc], two_sum(p, s)));
  }
  slots[t.slot_off + si] = y.hi;
  slots_lo[t.slot_off + si] = y.lo;
}

// Removing an element's rigid motion (exact for the products: K_s annihilates
// rigid motions, its FP64 rounding does not, and a region joined to the
// supports through void material moves rigidly by ~1e9 times its
// deformation).  The rigid motion (a - th y, b + th x) takes the element
// vector's values at DOF 0 (vertex (0,0) x), 1 (its y) and 3 (vertex (1,0)
// y); only the four vertex functions carry it.  For local DOF `row` of an
// order-P element with value xv, x0 = value of DOF 0, x1 = of DOF 1,
// th = x3 - x1: the deformation part, formed as the difference of nearby
// values first ((xv - x0) and x3 - x1 are exact when the values are within a
// factor 2 of each other), so its rounding is relative to the deformation,
// not to the rigid motion.  Non-vertex DOFs are returned unchanged.
template <int P>
__device__ __forceinline__ double rigid_free(double xv, int row, double x0, double x1, double th) {
  const int a = row >> 1, i = a % (P + 1), j = a / (P + 1);
  if (i > 1 || j > 1) return xv;
  return (row & 1) ? (xv - x1) - th * i : (xv - x0) + th * j;
}

// ---------------------------------------------------------------------------
// Element contraction on MFMA.  One block per tile of 16*NC element columns
// of one system; the block's KS waves split the density cells of the
// reduction (wave w takes cells [w S / KS, (w+1) S / KS)) and their partial
// products are summed through LDS.  The tile's u_e (or p_old and z in PCG
// mode) are gathered once into LDS by the whole block, while wave 0 reduces
// the PCG scalars.
template <int P, int NC>
__global__ __launch_bounds__(512) void k_elem_mfma(GroupDev g, const Tile* __restrict__ tiles,
                                                  const double* __restrict__ E, const double* __restrict__ xin,
                                                  PcgDev s, int mode, int it_k) {
  constexpr int NE = ne_of(P), NEP = nep_of(P), MB = mb_of(P), NJ = NEP / 4, TC = 16 * NC;
  constexpr int NACC = MB * NC * 4;
  extern __shared__ double lds[];
  double* ush = lds + 2;             // [NEP][TC] (u or p_old), then [NEP][TC] z in PCG mode
  double* red = lds + 2;             // reused after the gather: [KS-1][NACC][64]
  const int ks = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const Tile t = tiles[g.tile_begin + xcd_tile(blockIdx.x, g.n_tiles, g.xcd_run)];
  // a stopped system has nothing to do (PCG mode also checks this iteration's residual below)
  if (mode != ELEM_APPLY && s.status[t.sys] != SYS_RUNNING) return;
  const bool pcg = mode == ELEM_PCG;
  const int n = lane & 15, kq = lane >> 4;
  // Everything that depends only on the tile is requested before the gather
  // barrier, so these loads overlap the gather: cell offsets, the scatter
  // slots (wave 0 stores), the first density cell's A fragments and moduli.
  int cellb[NC];
  bool valid[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = c * 16 + n;
    valid[c] = col < t.count;
    cellb[c] = valid[c] ? g.cell[t.elem_begin + col] : 0;
  }
  int sidx[NC][MB][4];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = b * 16 + kq + 4 * r;
        sidx[c][b][r] = (wave == 0 && valid[c] && row < NE) ? g.sidx[row * g.npad + t.elem_begin + c * 16 + n] : -1;
      }
  const int s_begin = (wave * g.S) / ks, s_end = ((wave + 1) * g.S) / ks;
  const double* __restrict__ kf = g.kfrag + lane;
  // One density cell's A fragments (NJ k-steps x MB row blocks) and moduli.
  auto load_slice = [&](int sc, double (&a)[NJ][MB], double (&e)[NC]) {
    const double* __restrict__ kfs = kf + (size_t)sc * NJ * MB * 64;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
      for (int b = 0; b < MB; ++b) a[jj][b] = kfs[(jj * MB + b) * 64];
#pragma unroll
    for (int c = 0; c < NC; ++c) e[c] = valid[c] ? E[cellb[c] + sc] : 0.0;
  };
  double a0[NJ][MB], e0[NC];
  if (s_begin < s_end) load_slice(s_begin, a0, e0);

  if (pcg && wave == 0) {
    const Scal sc = pcg_state(s, t.sys, t.pc_begin, t.pc_end, *s.it_base + it_k, true);
    if (lane == 0) {
      lds[0] = sc.beta;
      lds[1] = sc.active ? 1.0 : 0.0;
    }
  }
  {
    // GU entries per thread at a time: their index loads, then their value
    // loads, all unconditional (clamped: column to the tile's last element,
    // DOF to the system's first, which every system has), so each group of
    // entries costs two memory round trips rather than two per entry
    constexpr int GU = 4, NT = NEP * TC;
    const double* __restrict__ xs = xin + t.dof_off;
    const double* __restrict__ zs = s.z + t.dof_off;
    for (int k0 = threadIdx.x; k0 < NT; k0 += GU * blockDim.x) {
      int gi[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int k = k0 + u * blockDim.x;
        const int kc = k < NT ? k : NT - 1;
        const int row = kc / TC, col = kc - row * TC;
        const int gl = g.gidx[row * g.npad + t.elem_begin + (col < t.count ? col : t.count - 1)];
        gi[u] = (k < NT && col < t.count) ? gl : -1;
      }
      double v[GU], zv[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int gc = gi[u] >= 0 ? gi[u] : 0;
        const double xv = xs[gc];
        v[u] = gi[u] >= 0 ? xv : 0.0;
        zv[u] = 0.0;
        if (pcg) {
          const double zz = zs[gc];
          zv[u] = gi[u] >= 0 ? zz : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int k = k0 + u * blockDim.x;
        if (k < NT) {
          ush[k] = v[u];
          if (pcg) ush[NT + k] = zv[u];
        }
      }
    }
  }
  __syncthreads();
  if (pcg && lds[1] == 0.0) return;  // system stopped: uniform over the block
  const double beta = pcg ? lds[0] : 0.0;
  double u[NC][NJ];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = c * 16 + n;
    // the element vector (p = z + beta p_old formed exactly as k_dof1 stores it), rigid motion removed
    auto val = [&](int row) {
      const int k = row * TC + col;
      return pcg ? fma(beta, ush[k], ush[NEP * TC + k]) : ush[k];
    };
    const double x0 = val(0), x1 = val(1), th = val(3) - x1;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) u[c][jj] = rigid_free<P>(val(4 * jj + kq), 4 * jj + kq, x0, x1, th);
  }
  d4 acc[MB][NC];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[b][c] = d4{0.0, 0.0, 0.0, 0.0};

  auto mma_slice = [&](const double (&a)[NJ][MB], const double (&e)[NC]) {
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double bv = e[c] * u[c][jj];
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[jj][b], bv, acc[b][c], 0, 0, 0);
      }
  };
  if constexpr (NJ * MB <= 20) {
    // ping-pong register buffers: the next cell's fragments load during the
    // current cell's MFMAs
    double a1[NJ][MB], e1[NC];
    for (int sc = s_begin; sc < s_end; sc += 2) {
      if (sc + 1 < s_end) load_slice(sc + 1, a1, e1);
      mma_slice(a0, e0);
      if (sc + 1 >= s_end) break;
      if (sc + 2 < s_end) load_slice(sc + 2, a0, e0);
      mma_slice(a1, e1);
    }
  } else {
    for (int sc = s_begin; sc < s_end; ++sc) {
      if (sc > s_begin) load_slice(sc, a0, e0);
      mma_slice(a0, e0);
    }
  }

  if (ks > 1) {
    __syncthreads();  // the gather buffer is reused for the partial products
    if (wave > 0) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[((wave - 1) * NACC + (b * NC + c) * 4 + r) * 64 + lane] = acc[b][c][r];
    }
    __syncthreads();
    if (wave > 0) return;
    for (int w = 1; w < ks; ++w)
#pragma unroll
      for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[b][c][r] += red[((w - 1) * NACC + (b * NC + c) * 4 + r) * 64 + lane];
  }

  double* __restrict__ sl = s.slots + t.slot_off;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (sidx[c][b][r] >= 0) sl[sidx[c][b][r]] = acc[b][c][r];
}

// ---------------------------------------------------------------------------
// Element contraction with the cell tables staged in LDS, for the groups whose
// tables are large (p >= 3, and every group in the fused launch): one block of
// 4 waves per tile of 64 NC element columns, wave w taking columns
// [16 NC w, 16 NC (w + 1)).  Every wave runs all density cells.  The tables of
// the next cell are loaded from L2 by the whole block into the other half of
// an LDS double buffer while the current cell's MFMAs run, so each table is
// read from L2 once per 64 NC columns (instead of once per 16 NC in
// k_elem_mfma) and from LDS by the four waves.  The gathered element vectors
// (p = z + beta p_old formed once, rigid motion removed as in k_elem_mfma) sit
// in LDS as well; each wave writes its own columns' slots.  For the orders
// with a vector-ALU tail (valu_tail: p = 2, 4) the last 2 rows are FMAs of
// each lane's B value with the 2 table entries of its reduction index,
// summed over the 4 lanes that share a column at the end, instead of a
// 16-row MFMA block of which 14 rows are padding.
// Copies the FR doubles of one cell's tables from global memory to LDS with
// the direct global-to-LDS loads of gfx950 (16 bytes per lane, no registers):
// 1 KB chunks, chunk k by wave k % 4; the caller waits on vmcnt before the
// barrier that publishes them.  src and dst are 16-byte aligned (FR is even).
template <int FR>
__device__ __forceinline__ void stage_tables(const double* __restrict__ src, double* dst, int wave, int lane) {
  constexpr int NCH = (FR + 127) / 128;
  for (int ch = wave; ch < NCH; ch += 4) {
    const int off = ch * 128 + 2 * lane;
    if (off < FR)  // lane l fills dst[ch * 128 + 2 l ..]
      __builtin_amdgcn_global_load_lds(src + off, (__attribute__((address_space(3))) void*)(dst + ch * 128), 16, 0, 0);
  }
}

template <int P, int NC>
__device__ __forceinline__ void elem_lds_tile(const GroupDev& g, const Tile& t, const double* __restrict__ E,
                                              const double* __restrict__ xin, const PcgDev& s, int mode, int it_k,
                                              double* lds) {
  constexpr int NE = ne_of(P), NEP = nep_of(P), NJ = NEP / 4, WC = 16 * NC, TC = 4 * WC;
  constexpr int MB = mbm_of(P), TR = tr_of(P), FRJ = frj_of(P);
  constexpr int FR = NJ * FRJ;             // doubles of one cell's tables
  constexpr int NT = NEP * TC, GPT = (NT + 255) / 256;  // gathered entries, per thread
  // LDS: two cell-table buffers; the element vectors overlay the second one
  // (and beyond) until they are in registers
  double* afr = lds;                // [2][FR]
  double* ush = lds + FR;           // [NEP][TC] element vectors
  double* scal = lds + (2 * FR > FR + NT ? 2 * FR : FR + NT);  // [2] beta, active
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // a stopped system has nothing to do (PCG mode also checks this iteration's residual below)
  if (mode != ELEM_APPLY && s.status[t.sys] != SYS_RUNNING) return;
  const bool pcg = mode == ELEM_PCG;
  const int n = lane & 15, kq = lane >> 4;
  const double* __restrict__ kf = g.kfrags;
  stage_tables<FR>(kf, afr, wave, lane);  // cell 0, in flight during the gather
  int cellb[NC];
  bool valid[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = wave * WC + c * 16 + n;
    valid[c] = col < t.count;
    cellb[c] = valid[c] ? g.cell[t.elem_begin + col] : 0;
  }
  // the element vectors: clamped, unconditional loads (column to the tile's
  // last element, DOF to the system's first), zeroed where absent
  double gv[GPT], gz[GPT];
  const double* __restrict__ xs = xin + t.dof_off;
  const double* __restrict__ zs = s.z + t.dof_off;
  {
    int gi[GPT];
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int e = tid + 256 * k;
      const int ec = e < NT ? e : NT - 1;
      const int row = ec / TC, col = ec - row * TC;
      const int gl = g.gidx[row * g.npad + t.elem_begin + (col < t.count ? col : t.count - 1)];
      gi[k] = (e < NT && col < t.count) ? gl : -1;
    }
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int gc = gi[k] >= 0 ? gi[k] : 0;
      const double xv = xs[gc];
      gv[k] = gi[k] >= 0 ? xv : 0.0;
      gz[k] = 0.0;
      if (pcg) {
        const double zz = zs[gc];
        gz[k] = gi[k] >= 0 ? zz : 0.0;
      }
    }
  }
  if (pcg && wave == 0) {
    const Scal sc = pcg_state(s, t.sys, t.pc_begin, t.pc_end, *s.it_base + it_k, true);
    if (lane == 0) {
      scal[0] = sc.beta;
      scal[1] = sc.active ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  if (pcg && scal[1] == 0.0) {  // system stopped: uniform over the block
    __builtin_amdgcn_s_waitcnt(0);  // no table copy outlives the block
    return;
  }
  const double beta = pcg ? scal[0] : 0.0;
#pragma unroll
  for (int k = 0; k < GPT; ++k) {  // p = z + beta p_old, formed as k_dof1 stores it
    const int e = tid + 256 * k;
    if (e < NT) ush[e] = pcg ? fma(beta, gv[k], gz[k]) : gv[k];
  }
  __builtin_amdgcn_s_waitcnt(0);  // this wave's share of cell 0's tables has landed
  __syncthreads();
  double u[NC][NJ];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = wave * WC + c * 16 + n;
    const double x0 = ush[col], x1 = ush[TC + col], th = ush[3 * TC + col] - x1;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) u[c][jj] = rigid_free<P>(ush[(4 * jj + kq) * TC + col], 4 * jj + kq, x0, x1, th);
  }
  __syncthreads();  // the element vectors are in registers: the second table buffer is free
  d4 acc[MB][NC];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[b][c] = d4{0.0, 0.0, 0.0, 0.0};
  double tacc[NC][TR > 0 ? TR : 1];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < TR; ++r) tacc[c][r] = 0.0;
  double e[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) e[c] = valid[c] ? E[cellb[c]] : 0.0;
  for (int sc = 0; sc < g.S; ++sc) {
    const double* __restrict__ cur = afr + (sc & 1) * FR;
    double* nxt = afr + ((sc + 1) & 1) * FR;
    const bool more = sc + 1 < g.S;
    double en[NC];
    if (more) {  // next cell: tables (straight to LDS) and moduli in flight during this cell's MFMAs
      stage_tables<FR>(kf + (size_t)(sc + 1) * FR, nxt, wave, lane);
#pragma unroll
      for (int c = 0; c < NC; ++c) en[c] = valid[c] ? E[cellb[c] + sc + 1] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      double a[MB];
#pragma unroll
      for (int b = 0; b < MB; ++b) a[b] = cur[jj * FRJ + b * 64 + lane];
      double ta[TR > 0 ? TR : 1];
#pragma unroll
      for (int r = 0; r < TR; ++r) ta[r] = cur[jj * FRJ + MB * 64 + kq * TR + r];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double bv = e[c] * u[c][jj];
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[b], bv, acc[b][c], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < TR; ++r) tacc[c][r] = fma(ta[r], bv, tacc[c][r]);
      }
    }
    if (more) {
#pragma unroll
      for (int c = 0; c < NC; ++c) e[c] = en[c];
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's share of the next cell's tables has landed
    __syncthreads();  // the next cell's tables are in; this cell's buffer may be overwritten
  }
  // the scatter slots, requested now (not held in registers through the loop)
  double* __restrict__ sl = s.slots + t.slot_off;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = wave * WC + c * 16 + n;
    int sidx[MB][4];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = b * 16 + kq + 4 * r;
        sidx[b][r] = (valid[c] && row < NE) ? g.sidx[row * g.npad + t.elem_begin + col] : -1;
      }
    const int sidt = (TR > 0 && valid[c] && kq < TR) ? g.sidx[(16 * MB + kq) * g.npad + t.elem_begin + col] : -1;
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (sidx[b][r] >= 0) sl[sidx[b][r]] = acc[b][c][r];
    if constexpr (TR > 0) {
      // tail rows: sum over the 4 lanes of each column ((a + b) + (c + d), the
      // same value in all four), lane kq writes row 16 MB + kq
      double mine = 0.0;
#pragma unroll
      for (int r = 0; r < TR; ++r) {
        double v = tacc[c][r];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (kq == r) mine = v;
      }
      if (sidt >= 0) sl[sidt] = mine;
    }
  }
}

template <int P, int NC>
__global__ __launch_bounds__(256) void k_elem_mfma_lds(GroupDev g, const Tile* __restrict__ tiles,
                                                      const double* __restrict__ E, const double* __restrict__ xin,
                                                      PcgDev s, int mode, int it_k) {
  extern __shared__ double lds[];
  const Tile t = tiles[g.lds_tile_begin + xcd_tile(blockIdx.x, g.lds_n_tiles, g.xcd_run)];
  elem_lds_tile<P, NC>(g, t, E, xin, s, mode, it_k, lds);
}

// The product of every (p, d) group in one launch: one block of 4 waves per
// tile of 64 element columns of the combined tile list (the groups ordered
// by decreasing work per tile, so the long tiles start first and the short
// ones fill in), each block running the LDS-staged contraction of its
// tile's group.
__global__ __launch_bounds__(256) void k_elem_fused(const GroupDev* __restrict__ groups,
                                                   const Tile* __restrict__ tiles, int tile_begin, int n_tiles,
                                                   int xcd_run, const double* __restrict__ E,
                                                   const double* __restrict__ xin, PcgDev s, int mode, int it_k) {
  extern __shared__ double lds[];
  const Tile t = tiles[tile_begin + xcd_tile(blockIdx.x, n_tiles, xcd_run)];
  const GroupDev g = groups[t.group];
  switch (g.p) {  // uniform over the block
    case 1: elem_lds_tile<1, 1>(g, t, E, xin, s, mode, it_k, lds); break;
    case 2: elem_lds_tile<2, 1>(g, t, E, xin, s, mode, it_k, lds); break;
    case 3: elem_lds_tile<3, 1>(g, t, E, xin, s, mode, it_k, lds); break;
    default: elem_lds_tile<4, 1>(g, t, E, xin, s, mode, it_k, lds); break;
  }
}

// ---------------------------------------------------------------------------
// Vertex-column product: slots += sum_s E_s K_s[:, V] dz_V for a correction dz
// that is nonzero only at vertex DOFs (V: the element's 8 vertex DOFs), which
// is what the coarse-grid correction of the V-cycle adds to z.  With the
// slots holding K z from before the correction this gives K z after it,
// without the full product: the reduction runs over S * 8 instead of
// S * NEP entries (two MFMA k-steps per cell, A = the vertex columns of K_s,
// kfragv [S][2][MB][64]).  One wave per 16 element columns (blockIdx.y picks
// the part of the tile); running systems only; dz's rigid motion removed as
// in the other products.
template <int P>
__device__ __forceinline__ int vertex_dof(int v) {  // v = 0..7: vertices (0,0), (1,0), (0,1), (1,1), x and y
  return v < 4 ? v : 2 * (P + 1) + (v - 4);
}

template <int P>
__global__ __launch_bounds__(64) void k_elem_vertex(GroupDev g, const Tile* __restrict__ tiles,
                                                   const double* __restrict__ E, const double* __restrict__ dz,
                                                   PcgDev s) {
  constexpr int NE = ne_of(P), MB = mb_of(P);
  const Tile t = tiles[g.tile_begin + blockIdx.x];
  const int c0 = blockIdx.y * 16;
  if (c0 >= t.count || s.status[t.sys] != SYS_RUNNING) return;  // uniform over the wave
  const int lane = threadIdx.x, n = lane & 15, kq = lane >> 4;
  const bool valid = c0 + n < t.count;
  const int el = t.elem_begin + c0 + (valid ? n : 0);
  // dz at vertex DOFs kq and 4 + kq of this lane's column
  double v[2];
#pragma unroll
  for (int jj = 0; jj < 2; ++jj) {
    const int gi = valid ? g.gidx[vertex_dof<P>(4 * jj + kq) * g.npad + el] : -1;
    const double x = dz[t.dof_off + (gi >= 0 ? gi : 0)];
    v[jj] = gi >= 0 ? x : 0.0;
  }
  {  // rigid motion through DOFs 0, 1 (vertex (0,0)) and 3 (vertex (1,0) y): lanes n, 16 + n, 48 + n
    const double x0 = __shfl(v[0], n), x1 = __shfl(v[0], 16 + n), th = __shfl(v[0], 48 + n) - x1;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) v[jj] = rigid_free<P>(v[jj], vertex_dof<P>(4 * jj + kq), x0, x1, th);
  }
  int sidx[MB][4];
  double old[MB][4];
  double* __restrict__ sl = s.slots + t.slot_off;
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = b * 16 + kq + 4 * r;
      sidx[b][r] = (valid && row < NE) ? g.sidx[row * g.npad + el] : -1;
      const double o = sl[sidx[b][r] >= 0 ? sidx[b][r] : 0];
      old[b][r] = sidx[b][r] >= 0 ? o : 0.0;
    }
  const int cb = valid ? g.cell[el] : 0;
  const double* __restrict__ kf = g.kfragv + lane;
  d4 acc[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) acc[b] = d4{old[b][0], old[b][1], old[b][2], old[b][3]};
  for (int sc = 0; sc < g.S; ++sc) {
    const double e = valid ? E[cb + sc] : 0.0;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const double bv = e * v[jj];
#pragma unroll
      for (int b = 0; b < MB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kf[(((size_t)sc * 2 + jj) * MB + b) * 64], bv, acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (sidx[b][r] >= 0) sl[sidx[b][r]] = acc[b][r];
}

// ---------------------------------------------------------------------------
// Stored element matrices.  For a group whose contraction costs more than
// reading its element matrix (p = 4, d = 5: 2 S n_e^2 = 125 kflop per column
// against 10.2 KB per element, shared by the element's load cases; FP64 MFMA
// on gfx950 sustains about 10 flop per byte of HBM), K_e = sum_s E_s K_s is
// assembled once per design (its packed upper triangle, element-major,
// asm_ntp_of(p) doubles per column) and each product reads it: the same
// operator, rounded once per entry instead of once per product.

__device__ __forceinline__ int packed_row_start(int ne, int a) { return a * ne - (a * (a - 1)) / 2; }

// K_e for EA consecutive element columns per block: each thread takes
// entries (a, b <= ...) of the packed triangle, reads K_s[a][b] once for all
// EA elements and accumulates E_s K_s[a][b] in the order of s.
constexpr int ASSEMBLE_EA = 16;
template <int P>
__global__ __launch_bounds__(256) void k_elem_assemble(GroupDev g, const double* __restrict__ E,
                                                       double* __restrict__ kst) {
  constexpr int NE = ne_of(P), NTP = asm_ntp_of(P), EA = ASSEMBLE_EA;
  __shared__ double es[EA][MTO_MAX_D * MTO_MAX_D];
  const int e0 = blockIdx.x * EA, cnt = min(EA, g.n_elems - e0);
  for (int i = threadIdx.x; i < EA * g.S; i += 256) {
    const int e = i / g.S, sc = i - e * g.S;
    es[e][sc] = e < cnt ? E[g.cell[e0 + e] + sc] : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NE * NE; idx += 256) {
    const int a = idx / NE, b = idx - a * NE;
    if (b < a) continue;
    const double* __restrict__ kab = g.ks + (int64_t)a * NE + b;
    double v[EA];
#pragma unroll
    for (int e = 0; e < EA; ++e) v[e] = 0.0;
    for (int sc = 0; sc < g.S; ++sc) {
      const double k = kab[(int64_t)sc * NE * NE];
#pragma unroll
      for (int e = 0; e < EA; ++e) v[e] = fma(es[e][sc], k, v[e]);
    }
    const int pi = packed_row_start(NE, a) + (b - a);
#pragma unroll
    for (int e = 0; e < EA; ++e)
      if (e < cnt) kst[(int64_t)(e0 + e) * NTP + pi] = v[e];
  }
}

// The product with stored element matrices: slots = K_e (x_e - rigid motion)
// for every system of an instance from one read of K_e.  One block of 256
// threads per tile of EB = asm_cols_of(P) element columns of an instance's
// first system (the tiles of the Schwarz application), thread (column c,
// row a) for the first NE EB threads.  The tile's triangles are one
// contiguous range, loaded with 16-byte loads and staged in LDS while the
// element vectors are gathered (PCG mode: p = z + beta p_old formed as
// k_dof1 stores it, beta and the running test of each system reduced by one
// wave each); row a then sums K_e(a, b) w_b in order of b, w the element
// vector with its rigid motion removed as in the contraction kernels.
constexpr int STORED_SYS = 4;  // systems per pass over a tile (one wave reduces each one's scalars)
template <int P>
__global__ __launch_bounds__(256) void k_elem_stored(GroupDev g, const Tile* __restrict__ tiles,
                                                     const double* __restrict__ xin, PcgDev s, int mode, int it_k) {
  constexpr int NE = ne_of(P), NTP = asm_ntp_of(P), EB = asm_cols_of(P);
  static_assert(NE * EB <= 256, "one thread per row and column");
  constexpr int NB2 = EB * NTP / 2, LPT = (NB2 + 255) / 256;
  __shared__ double2 ks2[NB2];
  __shared__ double vs[STORED_SYS][EB][NE];
  __shared__ double sbeta[STORED_SYS];
  __shared__ int sact[STORED_SYS];
  const double* ksh = (const double*)ks2;
  const Tile t = tiles[g.ms_tile_begin + blockIdx.x];
  const int nsys = t.pc_begin;  // the instance's systems follow its first one
  const bool pcg = mode == ELEM_PCG;
  if (mode != ELEM_APPLY) {  // nothing to do once every system has stopped (no matrix read)
    bool any = false;
    for (int l = 0; l < nsys; ++l) any |= s.status[t.sys + l] == SYS_RUNNING;
    if (!any) return;  // uniform over the block
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double2* __restrict__ src = (const double2*)(g.kst + (int64_t)t.elem_begin * NTP);
  const int nw = t.count * (NTP / 2);
  double2 stg[LPT];
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = tid + 256 * k;
    stg[k] = i < nw ? src[i] : double2{0.0, 0.0};
  }
  const int c = tid / NE, a = tid - c * NE;
  const bool act = c < EB && c < t.count;
  const int64_t col = t.elem_begin + (act ? c : 0);
  const int id = act ? g.gidx[a * (int64_t)g.npad + col] : -1;
  const int si = act ? g.sidx[a * (int64_t)g.npad + col] : -1;
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = tid + 256 * k;
    if (i < NB2) ks2[i] = stg[k];
  }
  const int ra = packed_row_start(NE, a) - a;
  const double* __restrict__ krow = ksh + (act ? c : 0) * NTP;
  for (int l0 = 0; l0 < nsys; l0 += STORED_SYS) {
    const int np = min(STORED_SYS, nsys - l0);
    if (wave < np) {  // this pass's systems: beta and whether each runs
      const int sys = t.sys + l0 + wave;
      bool run;
      double beta = 0.0;
      if (pcg) {
        const SysDesc& sd = s.sys[sys];
        const Scal sc = pcg_state(s, sys, sd.chunk_begin, sd.chunk_end, *s.it_base + it_k, true);
        run = sc.active;
        beta = sc.beta;
      } else {
        run = mode == ELEM_APPLY || s.status[sys] == SYS_RUNNING;
      }
      if (lane == 0) {
        sbeta[wave] = beta;
        sact[wave] = run ? 1 : 0;
      }
    }
    __syncthreads();  // the scalars (and, on the first pass, the matrices)
    if (act) {
#pragma unroll
      for (int l = 0; l < STORED_SYS; ++l) {
        if (l >= np) break;
        double x = 0.0;
        if (sact[l] && id >= 0) {
          const SysDesc& sd = s.sys[t.sys + l0 + l];
          const double xv = xin[sd.dof_off + id];
          x = pcg ? fma(sbeta[l], xv, s.z[sd.dof_off + id]) : xv;
        }
        vs[l][c][a] = x;
      }
    }
    __syncthreads();  // the element vectors
    if (act) {
      double acc[STORED_SYS] = {0.0, 0.0, 0.0, 0.0};
      double x0[STORED_SYS], x1[STORED_SYS], th[STORED_SYS];
#pragma unroll
      for (int l = 0; l < STORED_SYS; ++l) {
        x0[l] = vs[l][c][0];
        x1[l] = vs[l][c][1];
        th[l] = vs[l][c][3] - x1[l];
      }
      auto row = [&](auto nl) {
        constexpr int NL = decltype(nl)::value;
#pragma unroll 10
        for (int b = 0; b < NE; ++b) {
          const int cb = packed_row_start(NE, b) - b;
          const double e = krow[b < a ? cb + a : ra + b];
#pragma unroll
          for (int l = 0; l < NL; ++l) acc[l] = fma(e, rigid_free<P>(vs[l][c][b], b, x0[l], x1[l], th[l]), acc[l]);
        }
      };
      switch (np) {  // uniform over the block
        case 1: row(std::integral_constant<int, 1>{}); break;
        case 2: row(std::integral_constant<int, 2>{}); break;
        case 3: row(std::integral_constant<int, 3>{}); break;
        default: row(std::integral_constant<int, 4>{}); break;
      }
#pragma unroll
      for (int l = 0; l < STORED_SYS; ++l)
        if (l < np && sact[l] && si >= 0) s.slots[s.sys[t.sys + l0 + l].slot_off + si] = acc[l];
    }
    if (l0 + STORED_SYS < nsys) __syncthreads();  // vs and the scalars are rewritten by the next pass
  }
}

// ---------------------------------------------------------------------------
// Comparison path: one thread per element column, FP64 VALU, K_s read from
// memory.  Block = 64 threads = one tile (at most 64 columns).
template <int P>
__global__ __launch_bounds__(64) void k_elem_plain(GroupDev g, const Tile* __restrict__ tiles,
                                                  const double* __restrict__ E, const double* __restrict__ xin,
                                                  PcgDev s, int mode, int it_k) {
  constexpr int NE = ne_of(P);
  const int tix = blockIdx.x;
  if (tix >= g.n_tiles) return;
  const Tile t = tiles[g.tile_begin + tix];
  if (mode == ELEM_APPLY_RUNNING && s.status[t.sys] != SYS_RUNNING) return;
  double beta = 0.0;
  if (mode == ELEM_PCG) {
    const Scal sc = pcg_state(s, t.sys, t.pc_begin, t.pc_end, *s.it_base + it_k, true);
    if (!sc.active) return;
    beta = sc.beta;
  }
  const int col = threadIdx.x;
  if (col >= t.count) return;
  const int el = t.elem_begin + col;
  const double* __restrict__ xs = xin + t.dof_off;
  const double* __restrict__ zs = s.z + t.dof_off;
  double u[NE];
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    const int gi = g.gidx[j * g.npad + el];
    double v = 0.0;
    if (gi >= 0) v = (mode == ELEM_PCG) ? fma(beta, xs[gi], zs[gi]) : xs[gi];
    u[j] = v;
  }
  {  // rigid motion removed (see rigid_free)
    const double x0 = u[0], x1 = u[1], th = u[3] - u[1];
#pragma unroll
    for (int j = 0; j < NE; ++j) u[j] = rigid_free<P>(u[j], j, x0, x1, th);
  }
  const int cb = g.cell[el];
  double* __restrict__ sl = s.slots + t.slot_off;
  for (int row = 0; row < NE; ++row) {
    double y = 0.0;
    for (int sc = 0; sc < g.S; ++sc) {
      const double* __restrict__ kr = g.ks + ((size_t)sc * NE + row) * NE;
      double tacc = 0.0;
#pragma unroll
      for (int j = 0; j < NE; ++j) tacc = fma(kr[j], u[j], tacc);
      y = fma(E[cb + sc], tacc, y);
    }
    const int si = g.sidx[row * g.npad + el];
    if (si >= 0) sl[si] = y;
  }
}

// ---------------------------------------------------------------------------
// Sensitivity: w_{e,s} = lam_e^T K_s u_e (lam = u for compliance) with K_s u_e on MFMA (same A fragments
// as the matvec), then a segmented dot over the rows each lane holds and a
// 4-lane butterfly; g = -E'(rho) w.  Both element vectors have their rigid
// motions (through DOFs 0, 1 and 3) removed first, as in k_elem_dd: K_s
// annihilates them exactly, its FP64 rounding does not.
template <int P, int NC>
__global__ __launch_bounds__(BLOCK) void k_sens_mfma(GroupDev g, const Tile* __restrict__ tiles,
                                                    const double* __restrict__ dE, const double* __restrict__ x,
                                                    const double* __restrict__ y, double* __restrict__ gout,
                                                    const SysDesc* __restrict__ sys) {
  constexpr int NEP = nep_of(P), MB = mb_of(P), NJ = NEP / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tix = blockIdx.x * WAVES + wave;
  if (tix >= g.n_tiles) return;
  const Tile t = tiles[g.tile_begin + tix];
  const SysDesc& sd = sys[t.sys];
  const int n = lane & 15, kq = lane >> 4;
  const double* __restrict__ xs = x + t.dof_off;
  const double* __restrict__ ys = y + t.dof_off;
  double u[NC][NJ], lm[NC][NJ];
  int cellb[NC];
  bool valid[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = c * 16 + n;
    valid[c] = col < t.count;
    const int el = t.elem_begin + col;
    cellb[c] = valid[c] ? g.cell[el] : 0;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int gi = valid[c] ? g.gidx[(4 * jj + kq) * g.npad + el] : -1;
      u[c][jj] = gi >= 0 ? xs[gi] : 0.0;
      lm[c][jj] = gi >= 0 ? ys[gi] : 0.0;
    }
    // rows 0, 1, 3 of column n sit in lanes n, 16 + n, 48 + n (k-step 0)
    const double ua = __shfl(u[c][0], n), ub = __shfl(u[c][0], 16 + n), uth = __shfl(u[c][0], 48 + n) - ub;
    const double la = __shfl(lm[c][0], n), lb = __shfl(lm[c][0], 16 + n), lth = __shfl(lm[c][0], 48 + n) - lb;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      u[c][jj] = rigid_free<P>(u[c][jj], 4 * jj + kq, ua, ub, uth);
      lm[c][jj] = rigid_free<P>(lm[c][jj], 4 * jj + kq, la, lb, lth);
    }
  }
  const double* __restrict__ kf = g.kfrag + lane;
  for (int sc = 0; sc < g.S; ++sc) {
    d4 acc[MB][NC];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[b][c] = d4{0.0, 0.0, 0.0, 0.0};
    const double* __restrict__ kfs = kf + (size_t)sc * NJ * MB * 64;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      double a[MB];
#pragma unroll
      for (int b = 0; b < MB; ++b) a[b] = kfs[(jj * MB + b) * 64];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < MB; ++b)
          acc[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[b], u[c][jj], acc[b][c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double w = 0.0;
#pragma unroll
      for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int jr = 4 * b + r;  // row 16b + kq + 4r = 4 jr + kq, held in u[c][jr]
          if (jr < NJ) w = fma(lm[c][jr < NJ ? jr : 0], acc[b][c][r], w);
        }
      w += __shfl_xor(w, 16);
      w += __shfl_xor(w, 32);
      if (kq == 0 && valid[c]) {
        const int64_t cell = (int64_t)cellb[c] + sc;
        gout[sd.g_off + cell] = -dE[cell] * w;
      }
    }
  }
}

// Jacobi diagonal contributions: thread per element column of a load-0 system.
template <int P>
__global__ __launch_bounds__(64) void k_diag_elem(GroupDev g, const Tile* __restrict__ tiles,
                                                 const double* __restrict__ E, double* __restrict__ slots,
                                                 const SysDesc* __restrict__ sys, const double* __restrict__ table) {
  constexpr int NE = ne_of(P);
  const int tix = blockIdx.x;
  if (tix >= g.n_tiles) return;
  const Tile t = tiles[g.tile_begin + tix];
  const SysDesc& sd = sys[t.sys];
  if (sd.load != 0) return;
  const int col = threadIdx.x;
  if (col >= t.count) return;
  const int el = t.elem_begin + col;
  const int cb = g.cell[el];
  double* __restrict__ sl = slots + sd.slot_off;
  for (int row = 0; row < NE; ++row) {
    double dsum = 0.0;
    for (int sc = 0; sc < g.S; ++sc) dsum = fma(E[cb + sc], table[sc * NE + row], dsum);
    const int si = g.sidx[row * g.npad + el];
    if (si >= 0) sl[si] = dsum;
  }
}

// ---------------------------------------------------------------------------
// SIMP moduli (Sec. 2.2).  A density that is not finite or lies outside
// [0, 1] sets *bad (when given; every writer stores the same 1) and gets the
// modulus E0 and derivative 0, so the kernels that follow still see valid
// numbers while the solve reports the input as invalid.
__global__ void k_simp(const double* __restrict__ rho, double* __restrict__ E, double* __restrict__ dE, int64_t n,
                       double E0, double Emin, double q, int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = rho[i];
  if (!(r >= 0.0 && r <= 1.0)) {  // NaN fails both tests
    if (bad) *bad = 1;
    E[i] = E0;
    dE[i] = 0.0;
    return;
  }
  const double rq1 = pow(r, q - 1.0);
  E[i] = Emin + r * rq1 * (E0 - Emin);
  dE[i] = q * rq1 * (E0 - Emin);
}

__global__ void k_fill(double* __restrict__ a, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ __launch_bounds__(VBLOCK) void k_dinv(PcgDev s, double* __restrict__ dinv, double scale) {
  const Chunk ch = s.chunks[blockIdx.x];
  if (ch.load != 0) return;
  const double* __restrict__ sl = s.slots + ch.slot_off;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK) {
    const double kd = s.kspr ? s.kspr[ch.inst_free_off + i] : 0.0;
    dinv[ch.inst_free_off + i] = scale / (slot_sum(sl, i, ch.nfv, ch.nfe) + kd);
  }
}

__global__ __launch_bounds__(VBLOCK) void k_init(PcgDev s, int use_slots) {
  __shared__ double lds[VWAVES + 4];
  const Chunk ch = s.chunks[blockIdx.x];
  const int64_t o = ch.dof_off;
  const double* __restrict__ sl = s.slots + ch.slot_off;
  double arz = 0.0, arr = 0.0, aff = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK) {
    const double fi = s.f[o + i];
    const double ri = use_slots == 2 ? s.r[o + i] : (use_slots ? fi - slot_sum(sl, i, ch.nfv, ch.nfe) : fi);
    const double zi = s.dinv[ch.inst_free_off + i] * ri;
    s.r[o + i] = ri;
    s.z[o + i] = zi;
    s.p[o + i] = 0.0;
    arz = fma(ri, zi, arz);
    arr = fma(ri, ri, arr);
    aff = fma(fi, fi, aff);
  }
  arz = block_sum<VWAVES>(arz, lds);
  arr = block_sum<VWAVES>(arr, lds);
  aff = block_sum<VWAVES>(aff, lds);
  if (threadIdx.x == 0) {
    s.part_rz[blockIdx.x] = arz;
    s.part_rz[s.n_chunks + blockIdx.x] = 1.0;  // rz of iteration -1: unused (beta_0 = 0)
    s.part_rr[blockIdx.x] = arr;
    s.part_rr[s.n_chunks + blockIdx.x] = arr;
    s.part_xx[blockIdx.x] = 0.0;  // x = 0 at the start of a cycle
    s.part_xx[s.n_chunks + blockIdx.x] = 0.0;
    s.part_aux[blockIdx.x] = aff;
  }
}

// Start of a PCG cycle.  At a restart (iterative refinement) a system whose
// true residual already meets rtol stays stopped: its cycle would end at
// iteration 0 with x = 0, so skipping it leaves every result the same, and
// its double-double residual in the slots stays valid for the next cycle end.
__global__ __launch_bounds__(BLOCK) void k_sys_setup(PcgDev s, double rtol2, int restart) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // invalid densities (flagged by k_simp): no system runs
  const bool bad = s.bad_rho && *s.bad_rho != 0;
  for (int sys = wave; sys < s.n_sys; sys += WAVES) {
    const SysDesc& sd = s.sys[sys];
    const double ff = wave_sum(s.part_aux, sd.chunk_begin, sd.chunk_end);
    if (lane == 0) {
      const double tol2 = rtol2 * ff;
      const bool met = restart && s.sys_out[4 * sys + 2] <= tol2;  // NaN runs (and breaks down)
      const int32_t st = bad ? SYS_BADINPUT : met ? SYS_CONVERGED : SYS_RUNNING;
      s.tol2[sys] = tol2;
      s.status[sys] = st;
      s.iters[sys] = 0;
      s.rep_count[sys] = 0;
      if (st != SYS_CONVERGED) s.dd_ok[sys] = 0;
    }
  }
  if (threadIdx.x == 0) *s.it_base = 0;
}

// The vector kernels run one free DOF per thread (a chunk is BLOCK DOFs of
// one system).  Each issues its data loads before reducing the PCG scalars,
// so the two memory round trips overlap.
__global__ __launch_bounds__(VBLOCK) void k_dof1(PcgDev s, int it_k) {
  __shared__ double lds[VWAVES + 4];
  const Chunk ch = s.chunks[blockIdx.x];
  // a stopped system loads nothing (most of the batch, late in a solve)
  if (s.status[ch.sys] != SYS_RUNNING) return;
  const int i = ch.begin + threadIdx.x;
  const bool in = i < ch.end;
  const int64_t o = ch.dof_off;
  // the iteration counter first: the scalar sums' addresses depend on it, and
  // the memory counter retires in order
  const int it = *s.it_base + it_k;
  // loads at a clamped index, unconditional (a lane past the chunk's end
  // rereads its last DOF and stores nothing)
  const int ic = in ? i : ch.end - 1;
  double qi = 0.0, kd = 0.0;
  const double po = s.p[o + ic], zi = s.z[o + ic];
  if (s.kspr) kd = s.kspr[ch.inst_free_off + ic];  // ground springs: q += k p
  const SlotVals sv = slot_fetch(s.slots + ch.slot_off, ic, ch.nfv, ch.nfe);
  if (threadIdx.x < 64) {
    const Scal sc = pcg_state(s, ch.sys, ch.pc_begin, ch.pc_end, it, true);
    if (threadIdx.x == 0) {
      lds[VWAVES] = sc.beta;
      lds[VWAVES + 1] = sc.active ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  qi = slot_add(sv);  // added after the scalar loads were issued
  Scal sc;
  sc.beta = lds[VWAVES];
  sc.active = lds[VWAVES + 1] != 0.0;
  if (!sc.active) {
    if (blockIdx.x == ch.pc_begin && threadIdx.x == 0 && s.status[ch.sys] == SYS_RUNNING)
      s.status[ch.sys] = SYS_CONVERGED;
    return;
  }
  double acc = 0.0;
  if (in) {
    const double pi = fma(sc.beta, po, zi);
    qi = fma(kd, pi, qi);
    s.p[o + i] = pi;
    s.q[o + i] = qi;
    acc = pi * qi;
  }
  acc = block_sum<VWAVES>(acc, lds);
  if (threadIdx.x == 0) s.part_pq[blockIdx.x] = acc;
}

__global__ __launch_bounds__(VBLOCK) void k_dof2(PcgDev s, int it_k) {
  __shared__ double lds[VWAVES + 4];
  const Chunk ch = s.chunks[blockIdx.x];
  if (s.status[ch.sys] != SYS_RUNNING) return;  // a stopped system loads nothing
  const int i = ch.begin + threadIdx.x;
  const bool in = i < ch.end;
  const int64_t o = ch.dof_off;
  const int it = *s.it_base + it_k;  // first: the scalar sums' addresses depend on it
  const int par = it & 1;
  // loads at a clamped index, unconditional (a lane past the chunk's end
  // rereads its last DOF and stores nothing)
  const int ic = in ? i : ch.end - 1;
  const double xi = s.x[o + ic], pi_ = s.p[o + ic], qi = s.q[o + ic], ri = s.r[o + ic];
  const double di = s.dinv[ch.inst_free_off + ic];
  if (threadIdx.x < 64) {
    // r.r and |D x|^2 (convergence), r.z and p.q of this system in one pass
    const double* const arr[4] = {s.part_rr + par * s.n_chunks, s.part_rz + par * s.n_chunks, s.part_pq,
                                  s.part_xx + par * s.n_chunks};
    double out[4];
    wave_sum_n<4>(arr, ch.pc_begin, ch.pc_end, out);
    const double rr = out[0], rz = out[1], pq = out[2];
    const bool active = s.status[ch.sys] == SYS_RUNNING && !(rr <= stop_thr2(s, ch.sys, out[3]));
    if (threadIdx.x == 0) {
      lds[VWAVES] = rz;
      lds[VWAVES + 1] = pq;
      lds[VWAVES + 2] = active ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const double rz = lds[VWAVES], pq = lds[VWAVES + 1];
  if (lds[VWAVES + 2] == 0.0) return;
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    if (blockIdx.x == ch.pc_begin && threadIdx.x == 0) s.status[ch.sys] = SYS_BREAKDOWN;
    return;
  }
  const double alpha = rz / pq;
  double arz = 0.0, arr = 0.0, axx = 0.0;
  if (in) {
    const double xn = fma(alpha, pi_, xi);
    s.x[o + i] = xn;
    const double rn = fma(-alpha, qi, ri);
    s.r[o + i] = rn;
    if (s.z_jacobi) {
      const double zn = di * rn;
      s.z[o + i] = zn;
      arz = rn * zn;
    }
    arr = rn * rn;
    const double dx = xn / di;  // (D x)_i, D = diag(K) (dinv = 1 / diag, or its l1 variant)
    axx = dx * dx;
  }
  arz = block_sum<VWAVES>(arz, lds);
  arr = block_sum<VWAVES>(arr, lds);
  axx = block_sum<VWAVES>(axx, lds);
  if (threadIdx.x == 0) {
    if (s.z_jacobi) s.part_rz[(par ^ 1) * s.n_chunks + blockIdx.x] = arz;
    s.part_rr[(par ^ 1) * s.n_chunks + blockIdx.x] = arr;
    s.part_xx[(par ^ 1) * s.n_chunks + blockIdx.x] = axx;
    if (blockIdx.x == ch.pc_begin) s.iters[ch.sys] = it + 1;
  }
}

// End of a chunk of G iterations, in two launches: k_advance_sys, one wave
// per system, latches the systems that have stopped and leaves in
// sys_out[4 sys + 3] how far a running one is from stopping (rr / tol2 over
// the floor, or -1 once stopped); k_advance_fin then reports the number of
// running systems and the largest of those ratios, and advances it_base.
__global__ __launch_bounds__(BLOCK) void k_advance_sys(PcgDev s, int G) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int it_new = *s.it_base + G;
  for (int sys = blockIdx.x * WAVES + wave; sys < s.n_sys; sys += gridDim.x * WAVES) {
    const SysDesc& sd = s.sys[sys];
    const double* const arr[2] = {s.part_rr + (it_new & 1) * s.n_chunks, s.part_xx + (it_new & 1) * s.n_chunks};
    double out[2];
    wave_sum_n<2>(arr, sd.chunk_begin, sd.chunk_end, out);
    const double rr = out[0], thr = stop_thr2(s, sys, out[1]);
    if (lane == 0) {
      double far = -1.0;
      if (s.status[sys] == SYS_RUNNING) {
        if (rr <= thr)
          s.status[sys] = SYS_CONVERGED;
        else
          far = rr / thr;
      }
      s.sys_out[4 * sys + 3] = far;
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_advance_fin(PcgDev s, int G) {
  __shared__ int cnt[WAVES];
  __shared__ double far_w[WAVES];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int active = 0;
  double far = 0.0;  // largest rr / tol2 of a running system (how far it is from stopping)
  for (int sys = threadIdx.x; sys < s.n_sys; sys += BLOCK) {
    const double f = s.sys_out[4 * sys + 3];
    if (f >= 0.0) {
      ++active;
      far = fmax(far, f);
    }
  }
  for (int m = 32; m >= 1; m >>= 1) {
    active += __shfl_xor(active, m);
    far = fmax(far, __shfl_xor(far, m));
  }
  if (lane == 0) {
    cnt[wave] = active;
    far_w[wave] = far;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    double f = 0.0;
    for (int w = 0; w < WAVES; ++w) {
      tot += cnt[w];
      f = fmax(f, far_w[w]);
    }
    s.progress[0] = (double)tot;
    s.progress[1] = f;
    *s.it_base += G;
  }
}

// Iterative refinement: the solution is carried as xhi + xlo (double-double)
// and each PCG cycle's correction x is added exactly, then x restarts at 0.
__global__ __launch_bounds__(VBLOCK) void k_accumulate(PcgDev s, double* __restrict__ xhi,
                                                       double* __restrict__ xlo, const int32_t* __restrict__ skip) {
  const Chunk ch = s.chunks[blockIdx.x];
  if (skip && skip[ch.sys]) return;  // a system not being refined here
  const int64_t o = ch.dof_off;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK) {
    const dd_t v = dd_add(dd_t{xhi[o + i], xlo[o + i]}, dd_t{s.x[o + i], 0.0});
    xhi[o + i] = v.hi;
    xlo[o + i] = v.lo;
    s.x[o + i] = 0.0;
  }
}

// r = f - K x from double-double slots, rounded once; also writes r into the
// PCG residual (a restart continues from it) and the partial sums.
// f_i - (K x)_i for free DOF i of chunk ch from the double-double slots
// (sh, sl), ground springs from x = xhi + xlo; rounded once.
__device__ __forceinline__ double residual_dd_at(const PcgDev& s, const Chunk& ch, int i,
                                                 const double* __restrict__ sh, const double* __restrict__ sl,
                                                 const double* __restrict__ xhi, const double* __restrict__ xlo) {
  const int64_t o = ch.dof_off;
  int64_t base;
  int cnt;
  slot_range(i, ch.nfv, ch.nfe, base, cnt);
  dd_t y{sh[base], sl[base]};
  for (int k = 1; k < cnt; ++k) y = dd_add(y, dd_t{sh[base + k], sl[base + k]});
  if (s.kspr) y = dd_add(y, dd_scale(s.kspr[ch.inst_free_off + i], dd_t{xhi[o + i], xlo[o + i]}));
  return dd_add(dd_t{s.f[o + i], 0.0}, dd_t{-y.hi, -y.lo}).hi;
}

__global__ __launch_bounds__(VBLOCK) void k_residual_dd(PcgDev s, const double* __restrict__ slots_lo,
                                                        const double* __restrict__ xhi,
                                                        const double* __restrict__ xlo) {
  __shared__ double lds[VWAVES + 4];
  const Chunk ch = s.chunks[blockIdx.x];
  const int64_t o = ch.dof_off;
  const double* __restrict__ sh = s.slots + ch.slot_off;
  const double* __restrict__ sl = slots_lo + ch.slot_off;
  double afx = 0.0, ares = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK) {
    const double fi = s.f[o + i];
    const double r = residual_dd_at(s, ch, i, sh, sl, xhi, xlo);
    s.r[o + i] = r;
    afx = fma(fi, xhi[o + i], afx);
    ares = fma(r, r, ares);
  }
  afx = block_sum<VWAVES>(afx, lds);
  ares = block_sum<VWAVES>(ares, lds);
  if (threadIdx.x == 0) {
    s.part_aux[s.n_chunks + blockIdx.x] = afx;
    s.part_aux[2 * s.n_chunks + blockIdx.x] = ares;
  }
}

// Residual replacement inside a PCG cycle (van der Vorst and Ye's scheme).
// The recursive residual r drifts from f - K x by the rounding of the FP64
// products, about the cycle's floor 4 eps ||D x|| (stop_thr2).  Once |r| has
// come within REPLACE_MARGIN of that floor (the drift is then at most 1/1000
// of |r|, too little to disturb the recurrences), the system's correction x
// is folded into the refined solution, r is replaced by the double-double
// true residual of the result, and PCG continues with the same search
// direction: the floor restarts from x = 0, so the cycle can go on to rtol
// instead of stopping at the floor for a cold restart.  Systems already
// within rtol, or stopped, are left alone.
constexpr double REPLACE_MARGIN = 1000.0;
// At most this many replacements per system and cycle: a true residual that
// no longer falls (rtol below what the double-double residual resolves) then
// ends the cycle at the floor as before, and the restarts' stall test decides.
constexpr int REPLACE_MAX = 8;

// rep_skip[sys] = 0 for the systems to refine now, 1 for the others; from the
// sums of the partials that iteration it (= *it_base + it_k) just wrote.
__global__ __launch_bounds__(BLOCK) void k_replace_flag(PcgDev s, int it_k) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int par = (*s.it_base + it_k + 1) & 1;
  for (int sys = blockIdx.x * WAVES + wave; sys < s.n_sys; sys += gridDim.x * WAVES) {  // one wave per system
    const SysDesc& sd = s.sys[sys];
    const double* const arr[2] = {s.part_rr + par * s.n_chunks, s.part_xx + par * s.n_chunks};
    double out[2];
    wave_sum_n<2>(arr, sd.chunk_begin, sd.chunk_end, out);
    const double rr = out[0];
    const double floor2 = 16.0 * 0x1p-106 * out[1];
    const bool rep = s.status[sys] == SYS_RUNNING && rr > s.tol2[sys] &&
                     rr <= REPLACE_MARGIN * REPLACE_MARGIN * floor2 && s.rep_count[sys] < REPLACE_MAX;
    if (lane == 0) {
      s.rep_skip[sys] = rep ? 0 : 1;
      if (rep) ++s.rep_count[sys];
    }
  }
}

// r = f - K x (x now the refined solution) for the flagged systems, with the
// partial sums the next iteration reads: r.r, |D x|^2 = 0 (the correction
// restarts from 0) and, where the iteration forms z = dinv r itself, z and r.z.
__global__ __launch_bounds__(VBLOCK) void k_residual_replace(PcgDev s, const double* __restrict__ slots_lo,
                                                             const double* __restrict__ xhi,
                                                             const double* __restrict__ xlo, int it_k) {
  __shared__ double lds[VWAVES + 4];
  const Chunk ch = s.chunks[blockIdx.x];
  if (s.rep_skip[ch.sys]) return;
  const int par = (*s.it_base + it_k + 1) & 1;
  const int64_t o = ch.dof_off;
  const double* __restrict__ sh = s.slots + ch.slot_off;
  const double* __restrict__ sl = slots_lo + ch.slot_off;
  double arr = 0.0, arz = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK) {
    const double r = residual_dd_at(s, ch, i, sh, sl, xhi, xlo);
    s.r[o + i] = r;
    arr = fma(r, r, arr);
    if (s.z_jacobi) {
      const double z = s.dinv[ch.inst_free_off + i] * r;
      s.z[o + i] = z;
      arz = fma(r, z, arz);
    }
  }
  arr = block_sum<VWAVES>(arr, lds);
  arz = block_sum<VWAVES>(arz, lds);
  if (threadIdx.x == 0) {
    s.part_rr[par * s.n_chunks + blockIdx.x] = arr;
    s.part_xx[par * s.n_chunks + blockIdx.x] = 0.0;
    if (s.z_jacobi) s.part_rz[par * s.n_chunks + blockIdx.x] = arz;
  }
}

__global__ __launch_bounds__(BLOCK) void k_residual_sums(PcgDev s) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int sys = wave; sys < s.n_sys; sys += WAVES) {
    const SysDesc& sd = s.sys[sys];
    const double ff = wave_sum(s.part_aux, sd.chunk_begin, sd.chunk_end);
    const double fx = wave_sum(s.part_aux + s.n_chunks, sd.chunk_begin, sd.chunk_end);
    const double rs = wave_sum(s.part_aux + 2 * s.n_chunks, sd.chunk_begin, sd.chunk_end);
    if (lane == 0) {
      s.sys_out[4 * sys + 0] = ff;
      s.sys_out[4 * sys + 1] = fx;
      s.sys_out[4 * sys + 2] = rs;
      s.dd_ok[sys] = 1;
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_compliance(PcgDev s, double* __restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < s.n_sys) c[s.sys[i].c_index] = s.sys_out[4 * i + 1];
}

__global__ __launch_bounds__(VBLOCK) void k_assemble_full(PcgDev s, const int32_t* __restrict__ f2f,
                                                        double* __restrict__ y, int diag_mode) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  if (diag_mode && sd.load != 0) return;
  const int64_t yo = diag_mode ? sd.diag_off : sd.u_off;
  const double* __restrict__ sl = s.slots + sd.slot_off;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK) {
    double v = slot_sum(sl, i, sd.nfv, sd.nfe);
    if (s.kspr) {  // ground springs: the diagonal gets k, the product k x (x in q)
      const double kd = s.kspr[sd.inst_free_off + i];
      v = diag_mode ? v + kd : fma(kd, s.q[sd.dof_off + i], v);
    }
    y[yo + f2f[sd.inst_free_off + i]] = v;
  }
}

__global__ __launch_bounds__(VBLOCK) void k_gather_free(PcgDev s, const int32_t* __restrict__ f2f,
                                                      const double* __restrict__ u, double* __restrict__ xf) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK)
    xf[sd.dof_off + i] = u[sd.u_off + f2f[sd.inst_free_off + i]];
}

__global__ __launch_bounds__(VBLOCK) void k_scatter_full(PcgDev s, const int32_t* __restrict__ f2f,
                                                       const double* __restrict__ xf, double* __restrict__ u) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += VBLOCK)
    u[sd.u_off + f2f[sd.inst_free_off + i]] = xf[sd.dof_off + i];
}

// out[cell] = sum over the instance's load cases l of w[c_index(l)] g[l][cell]
// (the backward of densities -> compliances).  One thread per cell.
__global__ __launch_bounds__(BLOCK) void k_weighted_sens(const double* __restrict__ g, const double* __restrict__ w,
                                                        double* __restrict__ out, const int64_t* __restrict__ inst_cell_off,
                                                        const int64_t* __restrict__ inst_g_off,
                                                        const int32_t* __restrict__ inst_c_off,
                                                        const int32_t* __restrict__ inst_L, int n_inst, int64_t n_cells) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n_cells) return;
  int lo = 0, hi = n_inst - 1;  // instance containing the cell
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst_cell_off[mid] <= cell) lo = mid;
    else hi = mid - 1;
  }
  const int64_t local = cell - inst_cell_off[lo];
  const int64_t ncell = inst_cell_off[lo + 1] - inst_cell_off[lo];
  double acc = 0.0;
  for (int l = 0; l < inst_L[lo]; ++l) acc = fma(w[inst_c_off[lo] + l], g[inst_g_off[lo] + l * ncell + local], acc);
  out[cell] = acc;
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Launches kernel k; with events the launch carries them on its own dispatch
// packet, so they time exactly this kernel (no separate marker packets).
template <typename K, typename... Args>
void launch_timed(K k, dim3 grid, dim3 block, uint32_t lds, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                  Args... args) {
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(k, grid, block, lds, st, ev0, ev1, 0u, args...);
  else
    hipLaunchKernelGGL(k, grid, block, lds, st, args...);
}

template <int P>
void launch_elem_p(const GroupDev& g, int path, int ncol, const Tile* tiles, const double* E, const double* xin,
                   const PcgDev& s, int mode, int it_k, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (path == MTO_PATH_PLAIN) {
    launch_timed(k_elem_plain<P>, dim3(g.n_tiles), dim3(64), 0u, st, ev0, ev1, g, tiles, E, xin, s, mode, it_k);
    return;
  }
  if constexpr (P >= 3) {
    if (g.lds_nc > 0) {
      if (g.lds_n_tiles == 0) return;
      const uint32_t lds = (uint32_t)elem_lds_staged_bytes(P, g.lds_nc);
      if (g.lds_nc == 1)
        launch_timed(k_elem_mfma_lds<P, 1>, dim3(g.lds_n_tiles), dim3(256), lds, st, ev0, ev1, g, tiles, E, xin, s,
                     mode, it_k);
      else
        launch_timed(k_elem_mfma_lds<P, 2>, dim3(g.lds_n_tiles), dim3(256), lds, st, ev0, ev1, g, tiles, E, xin, s,
                     mode, it_k);
      return;
    }
  }
  const dim3 grid(g.n_tiles), block(64 * g.waves);
  const uint32_t lds = (uint32_t)elem_lds_bytes(P, ncol, g.waves);
  switch (ncol) {
    case 1: launch_timed(k_elem_mfma<P, 1>, grid, block, lds, st, ev0, ev1, g, tiles, E, xin, s, mode, it_k); break;
    case 2: launch_timed(k_elem_mfma<P, 2>, grid, block, lds, st, ev0, ev1, g, tiles, E, xin, s, mode, it_k); break;
    default: launch_timed(k_elem_mfma<P, 4>, grid, block, lds, st, ev0, ev1, g, tiles, E, xin, s, mode, it_k); break;
  }
}

template <int P>
void launch_sens_p(const GroupDev& g, int ncol, const Tile* tiles, const double* dE, const double* x,
                   const double* y, double* gout, const SysDesc* sys, hipStream_t st) {
  const dim3 grid(nblocks(g.n_tiles, WAVES)), block(BLOCK);
  switch (ncol) {
    case 1: hipLaunchKernelGGL((k_sens_mfma<P, 1>), grid, block, 0, st, g, tiles, dE, x, y, gout, sys); break;
    case 2: hipLaunchKernelGGL((k_sens_mfma<P, 2>), grid, block, 0, st, g, tiles, dE, x, y, gout, sys); break;
    default: hipLaunchKernelGGL((k_sens_mfma<P, 4>), grid, block, 0, st, g, tiles, dE, x, y, gout, sys); break;
  }
}

}  // namespace

void launch_elem(const GroupDev& g, int path, const Tile* tiles, const double* E, const double* xin,
                 const PcgDev& s, int mode, int it_k, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (g.n_tiles == 0) return;
  switch (g.p) {
    case 1: launch_elem_p<1>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st, ev0, ev1); break;
    case 2: launch_elem_p<2>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st, ev0, ev1); break;
    case 3: launch_elem_p<3>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st, ev0, ev1); break;
    default: launch_elem_p<4>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st, ev0, ev1); break;
  }
}

void launch_elem_fused(const GroupDev* groups, const Tile* tiles, int tile_begin, int n_tiles, int xcd_run,
                       size_t lds_bytes, const double* E, const double* xin, const PcgDev& s, int mode, int it_k,
                       hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (n_tiles == 0) return;
  launch_timed(k_elem_fused, dim3(n_tiles), dim3(256), (uint32_t)lds_bytes, st, ev0, ev1, groups, tiles, tile_begin,
               n_tiles, xcd_run, E, xin, s, mode, it_k);
}

void launch_elem_stored(const GroupDev& g, const Tile* tiles, const double* xin, const PcgDev& s, int mode, int it_k,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (g.ms_n_tiles == 0) return;
  const dim3 grid(g.ms_n_tiles), block(256);
  switch (g.p) {
    case 1: launch_timed(k_elem_stored<1>, grid, block, 0u, st, ev0, ev1, g, tiles, xin, s, mode, it_k); break;
    case 2: launch_timed(k_elem_stored<2>, grid, block, 0u, st, ev0, ev1, g, tiles, xin, s, mode, it_k); break;
    case 3: launch_timed(k_elem_stored<3>, grid, block, 0u, st, ev0, ev1, g, tiles, xin, s, mode, it_k); break;
    default: launch_timed(k_elem_stored<4>, grid, block, 0u, st, ev0, ev1, g, tiles, xin, s, mode, it_k); break;
  }
}

void launch_elem_assemble(const GroupDev& g, const double* E, double* kst, hipStream_t st) {
  if (g.n_elems == 0) return;
  const dim3 grid((g.n_elems + ASSEMBLE_EA - 1) / ASSEMBLE_EA), block(256);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_elem_assemble<1>, grid, block, 0, st, g, E, kst); break;
    case 2: hipLaunchKernelGGL(k_elem_assemble<2>, grid, block, 0, st, g, E, kst); break;
    case 3: hipLaunchKernelGGL(k_elem_assemble<3>, grid, block, 0, st, g, E, kst); break;
    default: hipLaunchKernelGGL(k_elem_assemble<4>, grid, block, 0, st, g, E, kst); break;
  }
}

void launch_elem_vertex(const GroupDev& g, const Tile* tiles, const double* E, const double* dz, const PcgDev& s,
                        hipStream_t st) {
  if (g.n_tiles == 0) return;
  const dim3 grid(g.n_tiles, g.ncol), block(64);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_elem_vertex<1>, grid, block, 0, st, g, tiles, E, dz, s); break;
    case 2: hipLaunchKernelGGL(k_elem_vertex<2>, grid, block, 0, st, g, tiles, E, dz, s); break;
    case 3: hipLaunchKernelGGL(k_elem_vertex<3>, grid, block, 0, st, g, tiles, E, dz, s); break;
    default: hipLaunchKernelGGL(k_elem_vertex<4>, grid, block, 0, st, g, tiles, E, dz, s); break;
  }
}

void launch_sens(const GroupDev& g, const Tile* tiles, const double* dE, const double* x, const double* y,
                 double* gout, const SysDesc* sys, hipStream_t st) {
  if (g.n_tiles == 0) return;
  switch (g.p) {
    case 1: launch_sens_p<1>(g, g.ncol, tiles, dE, x, y, gout, sys, st); break;
    case 2: launch_sens_p<2>(g, g.ncol, tiles, dE, x, y, gout, sys, st); break;
    case 3: launch_sens_p<3>(g, g.ncol, tiles, dE, x, y, gout, sys, st); break;
    default: launch_sens_p<4>(g, g.ncol, tiles, dE, x, y, gout, sys, st); break;
  }
}

void launch_diag_elem(const GroupDev& g, const Tile* tiles, const double* E, double* slots, const SysDesc* sys,
                      const double* table, hipStream_t st) {
  if (g.n_tiles == 0) return;
  const dim3 grid(g.n_tiles), block(64);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_diag_elem<1>, grid, block, 0, st, g, tiles, E, slots, sys, table); break;
    case 2: hipLaunchKernelGGL(k_diag_elem<2>, grid, block, 0, st, g, tiles, E, slots, sys, table); break;
    case 3: hipLaunchKernelGGL(k_diag_elem<3>, grid, block, 0, st, g, tiles, E, slots, sys, table); break;
    default: hipLaunchKernelGGL(k_diag_elem<4>, grid, block, 0, st, g, tiles, E, slots, sys, table); break;
  }
}

void launch_simp(const double* rho, double* E, double* dE, int64_t n, double E0, double Emin, double q,
                 hipStream_t st, int32_t* bad) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_simp, dim3(nblocks(n, BLOCK)), dim3(BLOCK), 0, st, rho, E, dE, n, E0, Emin, q, bad);
}

void launch_fill(double* a, double v, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n, BLOCK)), dim3(BLOCK), 0, st, a, v, n);
}

void launch_fill_i32(int32_t* a, int32_t v, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n, BLOCK)), dim3(BLOCK), 0, st, a, v, n);
}

void launch_dinv(const PcgDev& s, double* dinv, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_dinv, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, dinv, scale);
}

void launch_init(const PcgDev& s, int use_slots, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, use_slots);
}

void launch_sys_setup(const PcgDev& s, double rtol, int restart, hipStream_t st) {
  hipLaunchKernelGGL(k_sys_setup, dim3(1), dim3(BLOCK), 0, st, s, rtol * rtol, restart);
}

void launch_dof1(const PcgDev& s, int it_k, hipStream_t st) {
  hipLaunchKernelGGL(k_dof1, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, it_k);
}

void launch_dof2(const PcgDev& s, int it_k, hipStream_t st) {
  hipLaunchKernelGGL(k_dof2, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, it_k);
}

void launch_advance(const PcgDev& s, int G, hipStream_t st) {
  hipLaunchKernelGGL(k_advance_sys, dim3((s.n_sys + WAVES - 1) / WAVES), dim3(BLOCK), 0, st, s, G);
  hipLaunchKernelGGL(k_advance_fin, dim3(1), dim3(BLOCK), 0, st, s, G);
}

void launch_accumulate(const PcgDev& s, double* xhi, double* xlo, hipStream_t st) {
  hipLaunchKernelGGL(k_accumulate, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, xhi, xlo, nullptr);
}

namespace {
void launch_elem_dd(const GroupDev* groups, int n_groups, const Tile* tiles, const double* E, const PcgDev& s,
                    const double* xhi, const double* xlo, double* slots_lo, const int32_t* skip, hipStream_t st);
}

void launch_replace(const GroupDev* groups, int n_groups, const Tile* tiles, const double* E, const PcgDev& s,
                    double* xhi, double* xlo, double* slots_lo, int it_k, hipStream_t st) {
  hipLaunchKernelGGL(k_replace_flag, dim3((s.n_sys + WAVES - 1) / WAVES), dim3(BLOCK), 0, st, s, it_k);
  hipLaunchKernelGGL(k_accumulate, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, xhi, xlo, s.rep_skip);
  launch_elem_dd(groups, n_groups, tiles, E, s, xhi, xlo, slots_lo, s.rep_skip, st);
  hipLaunchKernelGGL(k_residual_replace, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, slots_lo, xhi, xlo, it_k);
}

void launch_residual_dd(const GroupDev* groups, int n_groups, const Tile* tiles, const double* E, const PcgDev& s,
                        const double* xhi, const double* xlo, double* slots_lo, hipStream_t st) {
  launch_elem_dd(groups, n_groups, tiles, E, s, xhi, xlo, slots_lo, s.dd_ok, st);
  hipLaunchKernelGGL(k_residual_dd, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, slots_lo, xhi, xlo);
  hipLaunchKernelGGL(k_residual_sums, dim3(1), dim3(BLOCK), 0, st, s);
}

namespace {
// the double-double element products of every group, skipping the tiles of
// systems with skip[sys] != 0
void launch_elem_dd(const GroupDev* groups, int n_groups, const Tile* tiles, const double* E, const PcgDev& s,
                    const double* xhi, const double* xlo, double* slots_lo, const int32_t* skip, hipStream_t st) {
  for (int k = 0; k < n_groups; ++k) {
    const GroupDev& g = groups[k];
    if (g.n_tiles == 0) continue;
    const dim3 grid(g.n_tiles, g.ncol);  // tiles hold at most 16 ncol columns
    switch (g.p) {
      case 1:
        hipLaunchKernelGGL(k_elem_dd<1>, grid, dim3(16 * dd_rows<1>()), 0, st, g, tiles, E, xhi, xlo, s.slots, slots_lo, skip);
        break;
      case 2:
        hipLaunchKernelGGL(k_elem_dd<2>, grid, dim3(16 * dd_rows<2>()), 0, st, g, tiles, E, xhi, xlo, s.slots, slots_lo, skip);
        break;
      case 3:
        hipLaunchKernelGGL(k_elem_dd<3>, grid, dim3(16 * dd_rows<3>()), 0, st, g, tiles, E, xhi, xlo, s.slots, slots_lo, skip);
        break;
      default:
        hipLaunchKernelGGL(k_elem_dd<4>, grid, dim3(16 * dd_rows<4>()), 0, st, g, tiles, E, xhi, xlo, s.slots, slots_lo, skip);
        break;
    }
  }
}
}  // namespace


void launch_assemble_to_full(const PcgDev& s, const int32_t* free_to_full, double* yfull, int diag_mode,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_assemble_full, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, free_to_full, yfull, diag_mode);
}

void launch_gather_free(const PcgDev& s, const int32_t* free_to_full, const double* ufull, double* xfree,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_gather_free, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, free_to_full, ufull, xfree);
}

void launch_scatter_full(const PcgDev& s, const int32_t* free_to_full, const double* xfree, double* ufull,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_full, dim3(s.n_chunks), dim3(VBLOCK), 0, st, s, free_to_full, xfree, ufull);
}

void launch_weighted_sens(const double* g, const double* w, double* out, const int64_t* inst_cell_off,
                          const int64_t* inst_g_off, const int32_t* inst_c_off, const int32_t* inst_L, int n_inst,
                          int64_t n_cells, hipStream_t st) {
  if (n_cells == 0) return;
  hipLaunchKernelGGL(k_weighted_sens, dim3(nblocks(n_cells, BLOCK)), dim3(BLOCK), 0, st, g, w, out, inst_cell_off,
                     inst_g_off, inst_c_off, inst_L, n_inst, n_cells);
}

void launch_compliance(const PcgDev& s, double* c, hipStream_t st) {
  hipLaunchKernelGGL(k_compliance, dim3(nblocks(s.n_sys, BLOCK)), dim3(BLOCK), 0, st, s, c);
}

}  // namespace mto
