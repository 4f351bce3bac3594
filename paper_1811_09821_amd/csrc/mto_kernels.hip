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

#include "mto_kernels.hpp"

namespace mto {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;

// Sum of arr[a..b) by one wave: strided sequential sums per lane, then a xor
// butterfly.  Every lane ends with the same bits, and so does every wave that
// calls it on the same range.
__device__ __forceinline__ double wave_sum(const double* __restrict__ arr, int a, int b) {
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int k = a + lane; k < b; k += 64) v += arr[k];
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Deterministic block sum (BLOCK threads), valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < WAVES; ++w) t += lds[w];
  return t;
}

struct Scal {
  bool active;
  double beta;
};

// Convergence state and beta of system `sys` at iteration `it` (see header
// comment).  A newly converged system is latched by the caller's designated
// thread.
__device__ __forceinline__ Scal pcg_state(const PcgDev& s, int sys, int it, bool want_beta) {
  const SysDesc& sd = s.sys[sys];
  const int pi = it & 1;
  const double rr = wave_sum(s.part_rr + pi * s.n_chunks, sd.chunk_begin, sd.chunk_end);
  Scal o;
  o.active = (s.status[sys] == SYS_RUNNING) && !(rr <= s.tol2[sys]);
  o.beta = 0.0;
  if (o.active && want_beta && it > 0) {
    const double rz_new = wave_sum(s.part_rz + pi * s.n_chunks, sd.chunk_begin, sd.chunk_end);
    const double rz_old = wave_sum(s.part_rz + (pi ^ 1) * s.n_chunks, sd.chunk_begin, sd.chunk_end);
    o.beta = rz_new / rz_old;
  }
  return o;
}

__device__ __forceinline__ void slot_range(int i, int nfv, int nfe, int64_t& base, int& cnt) {
  if (i < nfv) {
    base = 4 * (int64_t)i;
    cnt = 4;
  } else if (i < nfv + nfe) {
    base = 4 * (int64_t)nfv + 2 * (int64_t)(i - nfv);
    cnt = 2;
  } else {
    base = 4 * (int64_t)nfv + 2 * (int64_t)nfe + (i - nfv - nfe);
    cnt = 1;
  }
}

__device__ __forceinline__ double slot_sum(const double* __restrict__ sl, int i, int nfv, int nfe) {
  int64_t base;
  int cnt;
  slot_range(i, nfv, nfe, base, cnt);
  double q = sl[base];
  for (int k = 1; k < cnt; ++k) q += sl[base + k];
  return q;
}

// ---------------------------------------------------------------------------
// Element contraction on MFMA.  One wave per tile of 16*NC element columns of
// one system; block = 4 waves (independent tiles).
template <int P, int NC>
__global__ __launch_bounds__(BLOCK) void k_elem_mfma(GroupDev g, const Tile* __restrict__ tiles,
                                                    const double* __restrict__ E,
                                                    const double* __restrict__ xin, PcgDev s, int mode,
                                                    int it_k) {
  constexpr int NE = ne_of(P), NEP = nep_of(P), MB = mb_of(P), NJ = NEP / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tix = blockIdx.x * WAVES + wave;
  if (tix >= g.n_tiles) return;
  const Tile t = tiles[g.tile_begin + tix];
  const SysDesc& sd = s.sys[t.sys];
  double beta = 0.0;
  if (mode == ELEM_PCG) {
    const Scal sc = pcg_state(s, t.sys, *s.it_base + it_k, true);
    if (!sc.active) return;
    beta = sc.beta;
  }
  const int n = lane & 15, kq = lane >> 4;
  const double* __restrict__ xs = xin + sd.dof_off;
  const double* __restrict__ zs = s.z + sd.dof_off;

  double u[NC][NJ];
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
      double v = 0.0;
      if (gi >= 0) v = (mode == ELEM_PCG) ? fma(beta, xs[gi], zs[gi]) : xs[gi];
      u[c][jj] = v;
    }
  }

  d4 acc[MB][NC];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[b][c] = d4{0.0, 0.0, 0.0, 0.0};

  const double* __restrict__ kf = g.kfrag + lane;
  for (int sc = 0; sc < g.S; ++sc) {
    double Es[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Es[c] = valid[c] ? E[cellb[c] + sc] : 0.0;
    const double* __restrict__ kfs = kf + (size_t)sc * NJ * MB * 64;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      double a[MB];
#pragma unroll
      for (int b = 0; b < MB; ++b) a[b] = kfs[(jj * MB + b) * 64];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double bv = Es[c] * u[c][jj];
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[b], bv, acc[b][c], 0, 0, 0);
      }
    }
  }

  double* __restrict__ sl = s.slots + sd.slot_off;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!valid[c]) continue;
    const int el = t.elem_begin + c * 16 + n;
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = b * 16 + kq + 4 * r;
        if (row < NE) {
          const int si = g.sidx[row * g.npad + el];
          if (si >= 0) sl[si] = acc[b][c][r];
        }
      }
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
  const SysDesc& sd = s.sys[t.sys];
  double beta = 0.0;
  if (mode == ELEM_PCG) {
    const Scal sc = pcg_state(s, t.sys, *s.it_base + it_k, true);
    if (!sc.active) return;
    beta = sc.beta;
  }
  const int col = threadIdx.x;
  if (col >= t.count) return;
  const int el = t.elem_begin + col;
  const double* __restrict__ xs = xin + sd.dof_off;
  const double* __restrict__ zs = s.z + sd.dof_off;
  double u[NE];
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    const int gi = g.gidx[j * g.npad + el];
    double v = 0.0;
    if (gi >= 0) v = (mode == ELEM_PCG) ? fma(beta, xs[gi], zs[gi]) : xs[gi];
    u[j] = v;
  }
  const int cb = g.cell[el];
  double* __restrict__ sl = s.slots + sd.slot_off;
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
// Sensitivity: w_{e,s} = u_e^T K_s u_e with K_s u_e on MFMA (same A fragments
// as the matvec), then a segmented dot over the rows each lane holds and a
// 4-lane butterfly; g = -E'(rho) w.
template <int P, int NC>
__global__ __launch_bounds__(BLOCK) void k_sens_mfma(GroupDev g, const Tile* __restrict__ tiles,
                                                    const double* __restrict__ dE, const double* __restrict__ x,
                                                    double* __restrict__ gout, const SysDesc* __restrict__ sys) {
  constexpr int NEP = nep_of(P), MB = mb_of(P), NJ = NEP / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tix = blockIdx.x * WAVES + wave;
  if (tix >= g.n_tiles) return;
  const Tile t = tiles[g.tile_begin + tix];
  const SysDesc& sd = sys[t.sys];
  const int n = lane & 15, kq = lane >> 4;
  const double* __restrict__ xs = x + sd.dof_off;
  double u[NC][NJ];
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
          if (jr < NJ) w = fma(u[c][jr < NJ ? jr : 0], acc[b][c][r], w);
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
                                                 const SysDesc* __restrict__ sys) {
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
    for (int sc = 0; sc < g.S; ++sc) dsum = fma(E[cb + sc], g.kdiag[sc * NE + row], dsum);
    const int si = g.sidx[row * g.npad + el];
    if (si >= 0) sl[si] = dsum;
  }
}

// ---------------------------------------------------------------------------
__global__ void k_simp(const double* __restrict__ rho, double* __restrict__ E, double* __restrict__ dE, int64_t n,
                       double E0, double Emin, double q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = rho[i];
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

__global__ __launch_bounds__(BLOCK) void k_dinv(PcgDev s, double* __restrict__ dinv) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  if (sd.load != 0) return;
  const double* __restrict__ sl = s.slots + sd.slot_off;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK)
    dinv[sd.inst_free_off + i] = 1.0 / slot_sum(sl, i, sd.nfv, sd.nfe);
}

__global__ __launch_bounds__(BLOCK) void k_init(PcgDev s, int use_slots) {
  __shared__ double lds[WAVES];
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  const int64_t o = sd.dof_off;
  const double* __restrict__ sl = s.slots + sd.slot_off;
  double arz = 0.0, arr = 0.0, aff = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK) {
    const double fi = s.f[o + i];
    const double ri = use_slots ? fi - slot_sum(sl, i, sd.nfv, sd.nfe) : fi;
    const double zi = s.dinv[sd.inst_free_off + i] * ri;
    s.r[o + i] = ri;
    s.z[o + i] = zi;
    s.p[o + i] = 0.0;
    arz = fma(ri, zi, arz);
    arr = fma(ri, ri, arr);
    aff = fma(fi, fi, aff);
  }
  arz = block_sum(arz, lds);
  arr = block_sum(arr, lds);
  aff = block_sum(aff, lds);
  if (threadIdx.x == 0) {
    s.part_rz[blockIdx.x] = arz;
    s.part_rz[s.n_chunks + blockIdx.x] = 1.0;  // rz of iteration -1: unused (beta_0 = 0)
    s.part_rr[blockIdx.x] = arr;
    s.part_rr[s.n_chunks + blockIdx.x] = arr;
    s.part_aux[blockIdx.x] = aff;
  }
}

__global__ __launch_bounds__(BLOCK) void k_sys_setup(PcgDev s, double rtol2) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int sys = wave; sys < s.n_sys; sys += WAVES) {
    const SysDesc& sd = s.sys[sys];
    const double ff = wave_sum(s.part_aux, sd.chunk_begin, sd.chunk_end);
    if (lane == 0) {
      s.tol2[sys] = rtol2 * ff;
      s.status[sys] = SYS_RUNNING;
      s.iters[sys] = 0;
    }
  }
  if (threadIdx.x == 0) *s.it_base = 0;
}

__global__ __launch_bounds__(BLOCK) void k_dof1(PcgDev s, int it_k) {
  __shared__ double lds[WAVES];
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  const int it = *s.it_base + it_k;
  const Scal sc = pcg_state(s, ch.sys, it, true);
  if (!sc.active) {
    if (blockIdx.x == sd.chunk_begin && threadIdx.x == 0 && s.status[ch.sys] == SYS_RUNNING)
      s.status[ch.sys] = SYS_CONVERGED;
    return;
  }
  const int64_t o = sd.dof_off;
  const double* __restrict__ sl = s.slots + sd.slot_off;
  double acc = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK) {
    const double qi = slot_sum(sl, i, sd.nfv, sd.nfe);
    const double pi = fma(sc.beta, s.p[o + i], s.z[o + i]);
    s.p[o + i] = pi;
    s.q[o + i] = qi;
    acc = fma(pi, qi, acc);
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) s.part_pq[blockIdx.x] = acc;
}

__global__ __launch_bounds__(BLOCK) void k_dof2(PcgDev s, int it_k) {
  __shared__ double lds[WAVES];
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  const int it = *s.it_base + it_k;
  const Scal sc = pcg_state(s, ch.sys, it, false);
  if (!sc.active) return;
  const int pi = it & 1;
  const double rz = wave_sum(s.part_rz + pi * s.n_chunks, sd.chunk_begin, sd.chunk_end);
  const double pq = wave_sum(s.part_pq, sd.chunk_begin, sd.chunk_end);
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    if (blockIdx.x == sd.chunk_begin && threadIdx.x == 0) s.status[ch.sys] = SYS_BREAKDOWN;
    return;
  }
  const double alpha = rz / pq;
  const int64_t o = sd.dof_off;
  double arz = 0.0, arr = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK) {
    s.x[o + i] = fma(alpha, s.p[o + i], s.x[o + i]);
    const double ri = fma(-alpha, s.q[o + i], s.r[o + i]);
    const double zi = s.dinv[sd.inst_free_off + i] * ri;
    s.r[o + i] = ri;
    s.z[o + i] = zi;
    arz = fma(ri, zi, arz);
    arr = fma(ri, ri, arr);
  }
  arz = block_sum(arz, lds);
  arr = block_sum(arr, lds);
  if (threadIdx.x == 0) {
    s.part_rz[(pi ^ 1) * s.n_chunks + blockIdx.x] = arz;
    s.part_rr[(pi ^ 1) * s.n_chunks + blockIdx.x] = arr;
    if (blockIdx.x == sd.chunk_begin) s.iters[ch.sys] = it + 1;
  }
}

__global__ __launch_bounds__(BLOCK) void k_advance(PcgDev s, int G) {
  __shared__ int cnt[WAVES];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int it_new = *s.it_base + G;
  int active = 0;
  for (int sys = wave; sys < s.n_sys; sys += WAVES) {
    const SysDesc& sd = s.sys[sys];
    const double rr = wave_sum(s.part_rr + (it_new & 1) * s.n_chunks, sd.chunk_begin, sd.chunk_end);
    const int st = s.status[sys];
    if (st == SYS_RUNNING) {
      if (rr <= s.tol2[sys]) {
        if (lane == 0) s.status[sys] = SYS_CONVERGED;
      } else {
        ++active;
      }
    }
  }
  if (lane == 0) cnt[wave] = active;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < WAVES; ++w) tot += cnt[w];
    *s.n_active = tot;
    *s.it_base = it_new;
  }
}

__global__ __launch_bounds__(BLOCK) void k_residual_partials(PcgDev s) {
  __shared__ double lds[WAVES];
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  const int64_t o = sd.dof_off;
  const double* __restrict__ sl = s.slots + sd.slot_off;
  double afx = 0.0, ares = 0.0;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK) {
    const double fi = s.f[o + i];
    const double ri = fi - slot_sum(sl, i, sd.nfv, sd.nfe);
    afx = fma(fi, s.x[o + i], afx);
    ares = fma(ri, ri, ares);
  }
  afx = block_sum(afx, lds);
  ares = block_sum(ares, lds);
  if (threadIdx.x == 0) {
    s.part_aux[s.n_chunks + blockIdx.x] = afx;
    s.part_aux[2 * s.n_chunks + blockIdx.x] = ares;
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
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_compliance(PcgDev s, double* __restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < s.n_sys) c[s.sys[i].c_index] = s.sys_out[4 * i + 1];
}

__global__ __launch_bounds__(BLOCK) void k_assemble_full(PcgDev s, const int32_t* __restrict__ f2f,
                                                        double* __restrict__ y, int diag_mode) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  if (diag_mode && sd.load != 0) return;
  const int64_t yo = diag_mode ? sd.diag_off : sd.u_off;
  const double* __restrict__ sl = s.slots + sd.slot_off;
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK)
    y[yo + f2f[sd.inst_free_off + i]] = slot_sum(sl, i, sd.nfv, sd.nfe);
}

__global__ __launch_bounds__(BLOCK) void k_gather_free(PcgDev s, const int32_t* __restrict__ f2f,
                                                      const double* __restrict__ u, double* __restrict__ xf) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK)
    xf[sd.dof_off + i] = u[sd.u_off + f2f[sd.inst_free_off + i]];
}

__global__ __launch_bounds__(BLOCK) void k_scatter_full(PcgDev s, const int32_t* __restrict__ f2f,
                                                       const double* __restrict__ xf, double* __restrict__ u) {
  const Chunk ch = s.chunks[blockIdx.x];
  const SysDesc& sd = s.sys[ch.sys];
  for (int i = ch.begin + threadIdx.x; i < ch.end; i += BLOCK)
    u[sd.u_off + f2f[sd.inst_free_off + i]] = xf[sd.dof_off + i];
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int P>
void launch_elem_p(const GroupDev& g, int path, int ncol, const Tile* tiles, const double* E, const double* xin,
                   const PcgDev& s, int mode, int it_k, hipStream_t st) {
  if (path == MTO_PATH_PLAIN) {
    hipLaunchKernelGGL(k_elem_plain<P>, dim3(g.n_tiles), dim3(64), 0, st, g, tiles, E, xin, s, mode, it_k);
    return;
  }
  const dim3 grid(nblocks(g.n_tiles, WAVES)), block(BLOCK);
  switch (ncol) {
    case 1: hipLaunchKernelGGL((k_elem_mfma<P, 1>), grid, block, 0, st, g, tiles, E, xin, s, mode, it_k); break;
    case 2: hipLaunchKernelGGL((k_elem_mfma<P, 2>), grid, block, 0, st, g, tiles, E, xin, s, mode, it_k); break;
    default: hipLaunchKernelGGL((k_elem_mfma<P, 4>), grid, block, 0, st, g, tiles, E, xin, s, mode, it_k); break;
  }
}

template <int P>
void launch_sens_p(const GroupDev& g, int ncol, const Tile* tiles, const double* dE, const double* x, double* gout,
                   const SysDesc* sys, hipStream_t st) {
  const dim3 grid(nblocks(g.n_tiles, WAVES)), block(BLOCK);
  switch (ncol) {
    case 1: hipLaunchKernelGGL((k_sens_mfma<P, 1>), grid, block, 0, st, g, tiles, dE, x, gout, sys); break;
    case 2: hipLaunchKernelGGL((k_sens_mfma<P, 2>), grid, block, 0, st, g, tiles, dE, x, gout, sys); break;
    default: hipLaunchKernelGGL((k_sens_mfma<P, 4>), grid, block, 0, st, g, tiles, dE, x, gout, sys); break;
  }
}

}  // namespace

void launch_elem(const GroupDev& g, int path, const Tile* tiles, const double* E, const double* xin,
                 const PcgDev& s, int mode, int it_k, hipStream_t st) {
  if (g.n_tiles == 0) return;
  switch (g.p) {
    case 1: launch_elem_p<1>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st); break;
    case 2: launch_elem_p<2>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st); break;
    case 3: launch_elem_p<3>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st); break;
    default: launch_elem_p<4>(g, path, g.ncol, tiles, E, xin, s, mode, it_k, st); break;
  }
}

void launch_sens(const GroupDev& g, const Tile* tiles, const double* dE, const double* x, double* gout,
                 const SysDesc* sys, hipStream_t st) {
  if (g.n_tiles == 0) return;
  switch (g.p) {
    case 1: launch_sens_p<1>(g, g.ncol, tiles, dE, x, gout, sys, st); break;
    case 2: launch_sens_p<2>(g, g.ncol, tiles, dE, x, gout, sys, st); break;
    case 3: launch_sens_p<3>(g, g.ncol, tiles, dE, x, gout, sys, st); break;
    default: launch_sens_p<4>(g, g.ncol, tiles, dE, x, gout, sys, st); break;
  }
}

void launch_diag_elem(const GroupDev& g, const Tile* tiles, const double* E, double* slots, const SysDesc* sys,
                      hipStream_t st) {
  if (g.n_tiles == 0) return;
  const dim3 grid(g.n_tiles), block(64);
  switch (g.p) {
    case 1: hipLaunchKernelGGL(k_diag_elem<1>, grid, block, 0, st, g, tiles, E, slots, sys); break;
    case 2: hipLaunchKernelGGL(k_diag_elem<2>, grid, block, 0, st, g, tiles, E, slots, sys); break;
    case 3: hipLaunchKernelGGL(k_diag_elem<3>, grid, block, 0, st, g, tiles, E, slots, sys); break;
    default: hipLaunchKernelGGL(k_diag_elem<4>, grid, block, 0, st, g, tiles, E, slots, sys); break;
  }
}

void launch_simp(const double* rho, double* E, double* dE, int64_t n, double E0, double Emin, double q,
                 hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_simp, dim3(nblocks(n, BLOCK)), dim3(BLOCK), 0, st, rho, E, dE, n, E0, Emin, q);
}

void launch_fill(double* a, double v, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n, BLOCK)), dim3(BLOCK), 0, st, a, v, n);
}

void launch_fill_i32(int32_t* a, int32_t v, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n, BLOCK)), dim3(BLOCK), 0, st, a, v, n);
}

void launch_dinv(const PcgDev& s, double* dinv, hipStream_t st) {
  hipLaunchKernelGGL(k_dinv, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, dinv);
}

void launch_init(const PcgDev& s, int use_slots, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, use_slots);
}

void launch_sys_setup(const PcgDev& s, double rtol, hipStream_t st) {
  hipLaunchKernelGGL(k_sys_setup, dim3(1), dim3(BLOCK), 0, st, s, rtol * rtol);
}

void launch_dof1(const PcgDev& s, int it_k, hipStream_t st) {
  hipLaunchKernelGGL(k_dof1, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, it_k);
}

void launch_dof2(const PcgDev& s, int it_k, hipStream_t st) {
  hipLaunchKernelGGL(k_dof2, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, it_k);
}

void launch_advance(const PcgDev& s, int G, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(BLOCK), 0, st, s, G);
}

void launch_residual(const PcgDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_partials, dim3(s.n_chunks), dim3(BLOCK), 0, st, s);
  hipLaunchKernelGGL(k_residual_sums, dim3(1), dim3(BLOCK), 0, st, s);
}

void launch_assemble_to_full(const PcgDev& s, const int32_t* free_to_full, double* yfull, int diag_mode,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_assemble_full, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, free_to_full, yfull, diag_mode);
}

void launch_gather_free(const PcgDev& s, const int32_t* free_to_full, const double* ufull, double* xfree,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_gather_free, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, free_to_full, ufull, xfree);
}

void launch_scatter_full(const PcgDev& s, const int32_t* free_to_full, const double* xfree, double* ufull,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_full, dim3(s.n_chunks), dim3(BLOCK), 0, st, s, free_to_full, xfree, ufull);
}

void launch_compliance(const PcgDev& s, double* c, hipStream_t st) {
  hipLaunchKernelGGL(k_compliance, dim3(nblocks(s.n_sys, BLOCK)), dim3(BLOCK), 0, st, s, c);
}

}  // namespace mto
