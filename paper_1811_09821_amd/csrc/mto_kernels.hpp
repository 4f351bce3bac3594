// Launch interface of the HIP kernels (host side).  All pointers are device
// pointers; all launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include "mto_internal.hpp"

namespace mto {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on
// XCD i mod 8), each with its own L2.  These bijections of [0, T) keep
// neighbouring elements, which share vertex and edge DOFs in their gathers,
// in one L2.  run <= 0: each XCD takes one contiguous eighth of the tiles
// (best for a single system).  run > 0: each XCD takes runs of `run`
// consecutive tiles dealt round-robin, so that when the tiles of stopped
// systems return at once the remaining work is still spread over all XCDs
// (batches whose systems converge at different iterations).
__device__ __forceinline__ int xcd_tile(int i, int T, int run) {
  const int x = i & 7, k = i >> 3;
  if (run <= 0) {
    const int q = T >> 3, r = T & 7;
    return x * q + min(x, r) + k;
  }
  if (i >= T / (8 * run) * (8 * run)) return i;  // the tail, in order
  return ((k / run) * 8 + x) * run + k % run;
}

// Device view of one (p, d) element group.
struct GroupDev {
  int32_t p, d, S, npad;   // npad: stride of the DOF-major descriptor arrays
  int32_t n_elems;
  int32_t tile_begin, n_tiles, ncol;  // tiles of this group in the tile array
  int32_t waves;           // waves per tile (density-cell split of the reduction)
  int32_t xcd_run;         // tile order over the XCDs of the contraction (see xcd_tile)
  int32_t lds_nc;          // > 0: the contraction runs k_elem_mfma_lds<P, lds_nc> (p >= 3) on the
  int32_t lds_tile_begin;  //   tiles of 64 lds_nc columns [lds_tile_begin, + lds_n_tiles)
  int32_t lds_n_tiles;
  int32_t ms_tile_begin;   // tiles of the first system of every instance (asm_cols_of(p) columns), on
  int32_t ms_n_tiles;      //   which the Schwarz application serves all systems of the instance
  const double* kfrag;     // MFMA A fragments [S*NEP/4][MB][64]
  const double* kfrags;    // the LDS-staged contraction's tables [S][NEP/4][frj_of(p)] (staged_fragments)
  const double* kst;       // stored element matrices K_e (stored != 0): [npad][asm_ntp_of(p)] packed upper triangles
  int32_t stored;          // products of this group read kst (k_elem_stored) instead of contracting K_s
  const double* kfragv;    // the vertex columns of K_s as A fragments [S][2][MB][64] (vertex_fragments)
  const double* ks;        // plain K_s [S][ne][ne]
  const double* kdiag;     // diag(K_s) [S][ne]
  const double* kabs;      // row sums of |K_s| [S][ne] (l1 smoother)
  const int32_t* gidx;     // [NEP][npad] free DOF (instance-local) of local DOF, -1 absent
  const int32_t* sidx;     // [MB*16][npad] slot (instance-local), -1 absent
  const int32_t* msidx;    // [npad][ne][2]: (free DOF, slot) of local DOF a of column col at 2 (col ne + a),
                           //   -1 absent: the Schwarz application's gathers, one contiguous run per tile
  const int32_t* cell;     // [npad] first density cell (global)
};

// One (p, d) group for the QR-error indicator: order-(p+1) cell tables and
// the instance and element of every group column.
struct QrGroupDev {
  int32_t p, d, S, npad;
  int32_t n_elems;
  const double* tab;      // [S][NT] packed lower triangle of K_s^(p+1), (i, j <= i) at i (i+1)/2 + j
  const int32_t* gidx;    // as GroupDev::gidx
  const int32_t* cell;    // as GroupDev::cell
  const int32_t* eid;     // [n_elems] element index within its instance
  const int32_t* einst;   // [n_elems] instance
  double t[MTO_MAX_P + 1];  // 1D load transfer to the new order-(p+1) function (qr_load_transfer)
};

// Element lookup for the refinement indicators: element e of instance i is
// column el_col[el_base[i] + e] of group el_group[el_base[i] + e].
struct AdaptDev {
  const GroupDev* groups;
  const int32_t* el_group;
  const int32_t* el_col;
  const int32_t* nelx;       // per instance
  const int32_t* nely;
  const int64_t* el_base;    // per instance
  const int64_t* inst_eoff;  // per instance: offset of its [load case][element] block
};

// Bounds of the density indicator (Sec. 3.2.2) for one adaptive cycle.
struct DensityBounds {
  double rl, ru, cl, cu, avg;
};

// Slots of free DOF i of a system: 4 per vertex DOF, 2 per edge DOF, 1 per
// interior DOF, in that order.
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

// Assembled value of DOF i: its slots summed in a fixed order.
// Its slots are requested together (one memory round trip, not one per
// slot) by slot_fetch and added by slot_add in the order ((q0 + q1) + q2) + q3;
// a caller can put other loads between the two.
struct SlotVals {
  double q[4];
  int cnt;
};
__device__ __forceinline__ SlotVals slot_fetch(const double* __restrict__ sl, int i, int nfv, int nfe) {
  int64_t base;
  SlotVals v;
  slot_range(i, nfv, nfe, base, v.cnt);
  // unconditional loads (a slot past the DOF's count rereads its last one),
  // so no join waits for them; the unused values are zeroed after
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double x = sl[base + (k < v.cnt ? k : v.cnt - 1)];
    v.q[k] = k < v.cnt ? x : 0.0;
  }
  return v;
}
__device__ __forceinline__ double slot_add(const SlotVals& v) {
  const double q01 = v.q[0] + v.q[1];
  return v.cnt == 1 ? v.q[0] : (v.cnt == 2 ? q01 : (q01 + v.q[2]) + v.q[3]);
}
__device__ __forceinline__ double slot_sum(const double* __restrict__ sl, int i, int nfv, int nfe) {
  return slot_add(slot_fetch(sl, i, nfv, nfe));
}

// Iteration state shared by the PCG kernels.
struct PcgDev {
  const SysDesc* sys;
  const Chunk* chunks;
  int32_t n_chunks;
  int32_t n_sys;
  int32_t z_jacobi;        // 1: the iteration's vector update also forms z = dinv r and r.z (Jacobi and the
                           //   multigrid of Jacobi-type smoothing start from it); 0: the Schwarz V-cycle forms both
  double* x;
  double* r;
  double* z;
  double* p;
  double* q;
  const double* f;
  const double* dinv;      // per instance free DOF
  const double* kspr;      // per instance free DOF: ground-spring stiffness, or NULL (no springs)
  double* slots;
  double* part_pq;         // [n_chunks]
  double* part_rz;         // [2][n_chunks]
  double* part_rr;         // [2][n_chunks]
  double* part_xx;         // [2][n_chunks]: sum of (x_i / dinv_i)^2 (rounding floor of the cycle, see pcg_state)
  double* part_aux;        // [3][n_chunks]: f.f, f.x, |f - Kx|^2
  int32_t* status;         // [n_sys]
  int32_t* iters;          // [n_sys]
  double* tol2;            // [n_sys]
  double* sys_out;         // [n_sys][4]: f.f, f.x, |f-Kx|^2, and the last chunk's rr / tol2 of a running
                           //   system over its floor (-1: stopped; k_advance_sys)
  int32_t* dd_ok;          // [n_sys]: 1 while (slots, slots_lo) hold the double-double K x of the system's
                           //   refined solution (set with the true residual, cleared when the system runs)
  int32_t* rep_skip;       // [n_sys]: 0 for the systems whose residual is replaced at this point of the
                           //   cycle (k_replace_flag), 1 for the others
  int32_t* rep_count;      // [n_sys]: residual replacements in this cycle
  int32_t* it_base;        // [1]
  double* progress;        // [2]: systems still running, largest rr / tol2 among them
  const int32_t* bad_rho;  // [1] or NULL: set by k_simp for an invalid density
};

// ELEM_APPLY_RUNNING: as ELEM_APPLY, skipping systems whose PCG has stopped.
enum ElemMode { ELEM_APPLY = 0, ELEM_PCG = 1, ELEM_APPLY_RUNNING = 2 };

// Dynamic LDS of the MFMA element kernel: two scalars, then the larger of the
// gathered tile ([2][NEP][16 ncol] doubles) and the partial products of
// waves 1..ks-1 ([ks-1][MB * ncol * 4][64] doubles).
inline size_t elem_lds_bytes(int p, int ncol, int ks) {
  const size_t gather = 2 * (size_t)nep_of(p) * 16 * ncol;
  const size_t red = (size_t)(ks - 1) * mb_of(p) * ncol * 4 * 64;
  return 8 * (2 + (gather > red ? gather : red));
}
constexpr size_t ELEM_LDS_LIMIT = 64 * 1024;

// Dynamic LDS of the LDS-staged contraction k_elem_mfma_lds<P, nc>: the A
// fragments of two cells, the tile's 64 nc element vectors overlaying the
// second (and beyond, where larger), and two scalars.
inline size_t elem_lds_staged_bytes(int p, int nc) {
  const size_t fr = (size_t)(nep_of(p) / 4) * frj_of(p), nt = (size_t)nep_of(p) * 64 * nc;
  return 8 * ((2 * fr > fr + nt ? 2 * fr : fr + nt) + 2);
}
constexpr size_t ELEM_LDS_STAGED_LIMIT = 160 * 1024;

// y-slots of K applied to the vector `xin` (ELEM_APPLY) or to the PCG search
// direction p = z + beta p formed on the fly (ELEM_PCG), for the tiles of one group.
// Optional events ev0/ev1 record the start and end of this kernel itself.
void launch_elem(const GroupDev& g, int path, const Tile* tiles, const double* E, const double* xin,
                 const PcgDev& s, int mode, int it_k, hipStream_t st, hipEvent_t ev0 = nullptr,
                 hipEvent_t ev1 = nullptr);
// The product of every group in one launch (k_elem_fused): tiles
// [tile_begin, + n_tiles) of 64 columns from any group (Tile::group indexes
// the device array `groups`); lds_bytes: the largest elem_lds_staged_bytes(p, 1)
// of the groups.
void launch_elem_fused(const GroupDev* groups, const Tile* tiles, int tile_begin, int n_tiles, int xcd_run,
                       size_t lds_bytes, const double* E, const double* xin, const PcgDev& s, int mode, int it_k,
                       hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// K_e = sum_s E_s K_s of every column of the group, packed upper triangles
// [npad][asm_ntp_of(p)] (stored element matrices)
void launch_elem_assemble(const GroupDev& g, const double* E, double* kst, hipStream_t st);
// y-slots of the stored element matrices g.kst applied as launch_elem does
// (every system of each instance from one read of its matrices)
void launch_elem_stored(const GroupDev& g, const Tile* tiles, const double* xin, const PcgDev& s, int mode, int it_k,
                        hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// slots += K[:, vertex DOFs] dz for the running systems (dz in the free-DOF
// layout, read at vertex DOFs only; the slots hold K z before the call)
void launch_elem_vertex(const GroupDev& g, const Tile* tiles, const double* E, const double* dz, const PcgDev& s,
                        hipStream_t st);
// g = -E' lam_e^T K_s u_e per system, u from x and lam from y (free-DOF
// layout of the systems; y = x gives the compliance sensitivity)
void launch_sens(const GroupDev& g, const Tile* tiles, const double* dE, const double* x, const double* y,
                 double* gout, const SysDesc* sys, hipStream_t st);
// per element, sum_s E_s table[s][row] into the slots of load-0 systems
// (table = diag(K_s) for Jacobi, row sums of |K_s| for the l1 smoother)
void launch_diag_elem(const GroupDev& g, const Tile* tiles, const double* E, double* slots, const SysDesc* sys,
                      const double* table, hipStream_t st);

// E, E' of every cell (Sec. 2.2); bad (device int, may be NULL) is set to 1 if a
// density is not finite or outside [0, 1] (it is never cleared here)
void launch_simp(const double* rho, double* E, double* dE, int64_t n, double E0, double Emin, double q,
                 hipStream_t st, int32_t* bad = nullptr);
void launch_fill(double* a, double v, int64_t n, hipStream_t st);
void launch_fill_i32(int32_t* a, int32_t v, int64_t n, hipStream_t st);
// dinv = scale / (sum of slots) on the first system of each instance
void launch_dinv(const PcgDev& s, double* dinv, double scale, hipStream_t st);
// r = f (use_slots 0), f - assembled slots (1) or the r already stored (2);
// then z = dinv r, p = 0, partials
void launch_init(const PcgDev& s, int use_slots, hipStream_t st);
void launch_sys_setup(const PcgDev& s, double rtol, int restart, hipStream_t st);
void launch_dof1(const PcgDev& s, int it_k, hipStream_t st);
void launch_dof2(const PcgDev& s, int it_k, hipStream_t st);
void launch_advance(const PcgDev& s, int G, hipStream_t st);
// accurate true residual: double-double element contraction of xhi + xlo,
// then r = f - K x rounded once into the PCG residual, |r|^2 and f.xhi per system
// Residual replacement after iteration *it_base + it_k (before its V-cycle):
// flags the systems whose residual has come near the cycle's rounding floor,
// folds their correction into (xhi, xlo) and replaces r by the true residual.
void launch_replace(const GroupDev* groups, int n_groups, const Tile* tiles, const double* E, const PcgDev& s,
                    double* xhi, double* xlo, double* slots_lo, int it_k, hipStream_t st);
void launch_residual_dd(const GroupDev* groups, int n_groups, const Tile* tiles, const double* E, const PcgDev& s,
                        const double* xhi, const double* xlo, double* slots_lo, hipStream_t st);
// (xhi, xlo) += x exactly, then x = 0
void launch_accumulate(const PcgDev& s, double* xhi, double* xlo, hipStream_t st);
// assembled slots -> y in the u layout (zeros elsewhere must be pre-filled);
// diag_mode: only load-0 systems, at their per-instance offset diag_off
void launch_assemble_to_full(const PcgDev& s, const int32_t* free_to_full, double* yfull, int diag_mode,
                             hipStream_t st);
// x (free) <-> u layout
// QR-error indicator of every element of group g (see mto_qr.hip); x holds
// the displacements in the free-DOF layout of the systems.
void launch_qr(const QrGroupDev& g, const double* E, const double* x, const SysDesc* sys, const int32_t* inst_sys0,
               const int32_t* inst_L, const int64_t* inst_eoff, const int32_t* inst_nel, double* eps,
               hipStream_t st);
// Refinement indicators (see mto_adapt.hip): Gamma^a per (system, element)
// from displacements x in the free-DOF layout; Gamma^d per element.
void launch_kelly(const AdaptDev& a, const SysDesc* sys, int n_sys, int nel_max, const double* x, double* gamma,
                  hipStream_t st);
void launch_density_indicator(const AdaptDev& a, const double* rho, const DensityBounds& b, double* gamma,
                              int64_t n_el, hipStream_t st);
void launch_gather_free(const PcgDev& s, const int32_t* free_to_full, const double* ufull, double* xfree,
                        hipStream_t st);
void launch_scatter_full(const PcgDev& s, const int32_t* free_to_full, const double* xfree, double* ufull,
                         hipStream_t st);
void launch_compliance(const PcgDev& s, double* c, hipStream_t st);
// out = sum_l w_l g_l per instance (inst_cell_off has n_inst + 1 entries)
void launch_weighted_sens(const double* g, const double* w, double* out, const int64_t* inst_cell_off,
                          const int64_t* inst_g_off, const int32_t* inst_c_off, const int32_t* inst_L, int n_inst,
                          int64_t n_cells, hipStream_t st);

// ---- multigrid (mto_mg.hip) ----
void launch_mg_assemble1(const MgChunk* ch, int n, const MgElem* elems, const double* kv, const double* E,
                         const int32_t* vfree, double* A, double* mask, hipStream_t st);
void launch_mg_l1(const MgChunk* ch, int n, const double* A, double* dinv, hipStream_t st);
void launch_mg_rap(const MgChunk* ch, int n, double* A, double* mask, hipStream_t st);
// coarsest level of each instance: band Cholesky (one LDS-window block per
// instance) into band; then the dense inverse (band-order rows in scr),
// symmetrised into natural order in dense; nmax / bmax: largest DOF count and
// band width over the instances
void launch_mg_coarse_factor(const MgChunk* ch, int n, int bmax, const double* A, double* band, hipStream_t st);
void launch_mg_coarse_inverse(const MgChunk* ch, int n, int nmax, double* band, double* scr, double* dense,
                              hipStream_t st);
void launch_mg_restrict0(const MgChunk* ch, int n, const PcgDev& s, const int32_t* vfree, const double* dinv,
                         double* r1, double* e1, hipStream_t st);
// levels l-1 -> l of the V-cycle in one launch (ch: the level-l system chunks)
void launch_mg_resid_restrict(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* mask,
                              const double* dinv, double* r, double* e, hipStream_t st);
void launch_mg_coarse_solve(const MgChunk* ch, int n, int nmax, const PcgDev& s, const double* dense, const double* r,
                            double* e2, hipStream_t st);
// vfree != NULL (level 1): also z += e2 at the free vertex DOFs
void launch_mg_prolong_smooth(const MgChunk* ch, int n, const PcgDev& s, const double* A, const double* mask,
                              const double* dinv, const double* r, const double* e, double* e2, const int32_t* vfree,
                              hipStream_t st);
void launch_mg_prolong0(const MgChunk* ch, int n, const PcgDev& s, const int32_t* vfree, const double* e2,
                        hipStream_t st);
void launch_mg_post0(const PcgDev& s, int it_k, int init, hipStream_t st);

// ---- element-block additive Schwarz smoother (mto_mg.hip) ----
// Per element column of group `gi`: the assembled operator restricted to the
// element's free DOFs (own sum_s E_s K_s plus the shared-DOF entries of the
// eight neighbours), inverted; binv holds its upper triangle packed by rows,
// element-major: [npad][asm_ntp_of(p)] (the last entry of an odd count is
// padding), zero rows/columns at absent or supported DOFs.  groups: device array of all group views;
// nbr [8][npad]: global element index of each neighbour (-1: none);
// el_group / el_col: group and column of every global element.
void launch_asm_block(const GroupDev& g, int gi, const GroupDev* groups, const int32_t* nbr, const int32_t* el_group,
                      const int32_t* el_col, const double* E, double* binv, hipStream_t st);
// slots2 = omega * B_e v_e for the running systems of the group's tiles,
// with v_e gathered from v, or (resid) from v - assembled slots
void launch_asm_apply(const GroupDev& g, const Tile* tiles, const double* binv, const double* v, int resid,
                      const PcgDev& s, double* slots2, double omega, hipStream_t st);
// z = assembled slots2 (running systems)
void launch_asm_z(const PcgDev& s, const double* slots2, hipStream_t st);
// z += assembled slots2, partial sums of r.z (parity slot as k_mg_post0)
void launch_asm_post(const PcgDev& s, const double* slots2, int it_k, int init, hipStream_t st);

}  // namespace mto
