// Internal data structures shared by the host plan builder, the kernels and
// the C ABI.  Nothing here crosses the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mto.h"

namespace mto {

// Sizes of the element of order p: n_e = 2 (p+1)^2 local DOFs; NEP pads n_e
// to a multiple of 4 (the k-width of one f64 MFMA step) and MB counts the
// 16-row MFMA blocks that cover n_e output rows.
constexpr int ne_of(int p) { return 2 * (p + 1) * (p + 1); }
constexpr int nep_of(int p) { return (ne_of(p) + 3) / 4 * 4; }
constexpr int mb_of(int p) { return (ne_of(p) + 15) / 16; }
// Orders whose last row block would hold only 2 of its 16 rows (p = 2: 18
// rows, p = 4: 50 rows): the LDS-staged contraction runs the full 16-row
// blocks on MFMA and those last rows as FP64 FMAs on the vector ALU, which
// runs at the same FP64 rate as MFMA on gfx950 and overlaps it.
constexpr bool valu_tail(int p) { return ne_of(p) % 16 == 2 && ne_of(p) > 16; }
constexpr int mbm_of(int p) { return valu_tail(p) ? ne_of(p) / 16 : mb_of(p); }  // MFMA row blocks
constexpr int tr_of(int p) { return valu_tail(p) ? ne_of(p) % 16 : 0; }           // rows on the vector ALU
// Doubles per k-step of the LDS-staged contraction's tables (staged_fragments).
constexpr int frj_of(int p) { return mbm_of(p) * 64 + 4 * tr_of(p); }

// Element-block Schwarz smoother: the packed upper triangle of an element's
// block inverse, padded to an even count (so every element's triangle starts
// on 16 bytes), and the element columns per block of its application
// (NE rows each, at most 256 threads, the blocks' triangles staged in LDS).
constexpr int asm_ntp_of(int p) { return (ne_of(p) * (ne_of(p) + 1) / 2 + 1) / 2 * 2; }
constexpr int asm_cols_of(int p) { return p == 1 ? 32 : p == 2 ? 14 : p == 3 ? 8 : 4; }

// Host-side K_s tables of Appendix B's composite integration:
// ks[s*ne*ne + i*ne + j] for density cell s of a d x d grid.
std::vector<double> subcell_tables(int p, int d, double nu);

// Load transfer of the QR-error indicator (Sec. 3.2.3): the order-(p+1)
// element load integrates the order-p load field against the refined
// functions.  In 1D, with the hierarchic functions phi_0..phi_p of order p
// also the first p + 1 of order p + 1, the field with moments g (integrals
// against phi_0..phi_p) has moment t . g against the new function phi_{p+1},
// t = m_p^{-1} m[0..p][p+1] (m the unit-interval mass matrix).  The 2D
// transfer is the tensor product of the 1D one.  Returns t (p + 1 values).
std::vector<double> qr_load_transfer(int p);

// Rearranges K_s into the MFMA A-operand order: for k-step t (4 consecutive
// reduction indices k = s*NEP + j) and row block mb, lane l holds
// Kcat[mb*16 + l%16][4t + l/16], with Kcat[row][s*NEP + j] = K_s[row][j]
// (zero outside n_e).  Result length T*MB*64 with T = d*d*NEP/4.
std::vector<double> mfma_fragments(const std::vector<double>& ks, int p, int d);

// The tables of the LDS-staged contraction, [S][NEP/4][frj_of(p)]: for k-step
// jj of cell s, the A fragments of the mbm_of(p) MFMA row blocks as in
// mfma_fragments, then (valu_tail orders) the last tr_of(p) rows at the
// step's 4 reduction indices, [kq][r] = K_s[16 mbm + r][4 jj + kq] (zero
// beyond n_e).  Without a vector-ALU tail it equals mfma_fragments.
std::vector<double> staged_fragments(const std::vector<double>& ks, int p, int d);

// The columns of K_s at the element's 8 vertex DOFs (local DOFs 0..3 and
// 2(p+1)..2(p+1)+3, k = 0..7 in that order) as MFMA A operands: for k-step jj
// (k = 4 jj .. 4 jj + 3) and row block mb, lane l holds
// K_s[mb*16 + l%16][vertex DOF 4 jj + l/16] (zero past n_e).  Length S*2*MB*64.
std::vector<double> vertex_fragments(const std::vector<double>& ks, int p, int d);

// One design instance after numbering.
struct InstanceHost {
  int nelx = 0, nely = 0, L = 1;
  std::vector<int8_t> p, d;
  int64_t n_scalar = 0, n_dof = 0, n_cells = 0;
  std::vector<int64_t> cell_off;     // [nel+1]
  // free DOF numbering
  std::vector<int32_t> full_to_free; // [n_dof], -1 if supported
  std::vector<int32_t> free_to_full; // [n_free]
  int32_t n_free = 0, nfv = 0, nfe = 0, nfi = 0;  // free vertex / edge / interior DOFs
  int64_t n_slots = 0;
  // per element: free DOF and slot of each local DOF (-1: absent or supported)
  std::vector<int32_t> elem_free;    // [nel][ne(p_e)] packed by elem_dof_off
  std::vector<int32_t> elem_slot;
  std::vector<int64_t> elem_dof_off; // [nel+1]
  // loads: rhs per load case in the free numbering, [L][n_free]
  std::vector<double> f;
  // ground springs: (free DOF, stiffness)
  std::vector<std::pair<int32_t, double>> springs;
};

// The thread-local message behind mto_last_error (set_error returns code).
int set_error(int code, const std::string& msg);
void clear_error();

// Builds the numbering; returns MTO_OK or an error code with `err` filled.
int build_instance(const mto_problem& prob, InstanceHost& out, std::string& err);

// Per-iteration scalar state lives in partial-sum arrays; see the kernels.
// SYS_BADINPUT: a density of the solve was not finite or outside [0, 1].
enum SysStatus : int32_t { SYS_RUNNING = 0, SYS_CONVERGED = 1, SYS_BREAKDOWN = 2, SYS_BADINPUT = 3 };

// Descriptor of one tile of element columns: elements
// [elem_begin, elem_begin + count) of group `group`, all for system `sys`.
// The system's offsets and partial-sum range are copied in, so a kernel
// needs one descriptor load before its data loads.
struct Tile {
  int64_t dof_off;    // system offset in the PCG vectors
  int64_t slot_off;   // system offset in the slot array
  int32_t group;
  int32_t sys;
  int32_t elem_begin;
  int32_t count;
  int32_t pc_begin;   // the system's chunk (partial-sum) range; in the tiles of the Schwarz
  int32_t pc_end;     //   application (GroupDev::ms_*) pc_begin is the instance's number of systems
};

// A chunk of the free DOFs of one system for the vector kernels, with the
// system's constants copied in.
struct Chunk {
  int64_t dof_off;
  int64_t slot_off;
  int64_t inst_free_off;
  int32_t sys;
  int32_t begin;      // first DOF, relative to the system
  int32_t end;
  int32_t nfv, nfe;
  int32_t pc_begin;   // the system's chunk range
  int32_t pc_end;
  int32_t load;
};

// Per-system constants on the device.
struct SysDesc {
  int64_t dof_off;     // offset in the PCG vectors
  int64_t slot_off;    // offset in the slot array
  int64_t u_off;       // offset of this system's block of u
  int64_t g_off;       // offset of this system's block of g
  int64_t inst_free_off;  // offset of the instance's free DOFs (dinv, free_to_full)
  int64_t diag_off;    // offset of the instance in the per-instance (one load case) u layout
  int32_t n_free;
  int32_t nfv, nfe;
  int32_t chunk_begin, chunk_end;
  int32_t inst;
  int32_t load;
  int32_t c_index;     // index into c
};

// ---- geometric multigrid preconditioner (levels >= 1: vertex grids) ----

constexpr int MG_CHUNK = 256;      // nodes per level-kernel block
constexpr int MG_COARSE_MAX = 3000;  // DOFs of the coarsest grid (dense inverse from a band Cholesky)
constexpr int MG_BAND_MAX = 80;      // its band width: the Cholesky window of (b+9)(b+1) doubles and an
                                     // 8-column panel of (b+8) rows fit 64 KB of LDS
// Band factor storage per instance (n coarsest DOFs), zero outside the band:
//   row form    rows -MG_INV_PD .. n + MG_INV_PD - 1, stride MG_BAND_RS:
//               [t] = L[i][i - t] (t = 1 .. b), [128] = 1 / L[i][i]
//   column form columns 0 .. n + MG_INV_PD - 1, stride MG_BAND_CS:
//               [t] = L[j + 1 + t][j] (t = 0 .. b - 1), [127] = 1 / L[j][j]
// The padding lets the substitution kernels load two 64-entry runs per step
// without bounds tests (b < 64 + 64); the reciprocal diagonal sits where the
// run of the lane that finishes the row would otherwise read a zero.
constexpr int MG_INV_PD = 8;     // substitution steps whose factor entries are in flight
constexpr int MG_BAND_RS = 130;
constexpr int MG_BAND_CS = 128;
inline int64_t mg_band_doubles(int64_t n) {
  return (n + 2 * MG_INV_PD) * MG_BAND_RS + (n + MG_INV_PD) * MG_BAND_CS;
}

// Work unit of the level kernels: nodes [node_begin, node_end) of the level
// grid of one system (vector kernels) or one instance (operator kernels; sys
// is then -1).  Offsets are in nodes (vectors hold 2 DOFs per node, operators
// 36 doubles per node: nine 2 x 2 blocks).
struct MgChunk {
  int64_t vec, op;      // this level: system vector / instance operator node offsets
  int64_t fvec, fop;    // finer level (level >= 2)
  int64_t cvec, cop;    // coarser level (absent at the coarsest: -1)
  int64_t dense_off;    // coarsest level: offset of the instance's dense inverse
  int64_t band_off;     // coarsest level: offset of the instance's band Cholesky factor
  int64_t dof_off;      // level 1 only: the system's level-0 offsets
  int64_t slot_off;
  int64_t elem_off;     // level 1 only: the instance's first element in the MgElem table
  int32_t sys, inst;
  int32_t node_begin, node_end;
  int32_t nx, ny;       // this grid (elements per side)
  int32_t fnx, fny;     // finer grid (level >= 2)
  int32_t cnx, cny;     // coarser grid
  int32_t nfv, nfe;     // level 1 only: level-0 slot layout
  int32_t level;
  int32_t nsys;         // systems served from this chunk: 1 for a system chunk; in an instance-system
                        // chunk the instance's systems sys .. sys + nsys - 1, whose vectors follow each
                        // other (each the level's node count of the instance further on)
};

// Per instance element data for the level-1 (vertex-grid) assembly.
struct MgElem {
  int32_t cell_off;     // first density cell (global)
  int32_t kv_off;       // offset of its group's vertex-block table [S][4][4][2][2]
  int32_t S;
  int32_t pad;
};

}  // namespace mto
