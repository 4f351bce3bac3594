// Launch interface of the HIP kernels (host side).  All pointers are device
// pointers; all launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include "mto_internal.hpp"

namespace mto {

// Device view of one (p, d) element group.
struct GroupDev {
  int32_t p, d, S, npad;   // npad: stride of the DOF-major descriptor arrays
  int32_t n_elems;
  int32_t tile_begin, n_tiles, ncol;  // tiles of this group in the tile array
  const double* kfrag;     // MFMA A fragments [S*NEP/4][MB][64]
  const double* ks;        // plain K_s [S][ne][ne]
  const double* kdiag;     // diag(K_s) [S][ne]
  const int32_t* gidx;     // [NEP][npad] free DOF (instance-local) of local DOF, -1 absent
  const int32_t* sidx;     // [MB*16][npad] slot (instance-local), -1 absent
  const int32_t* cell;     // [npad] first density cell (global)
};

// Iteration state shared by the PCG kernels.
struct PcgDev {
  const SysDesc* sys;
  const Chunk* chunks;
  int32_t n_chunks;
  int32_t n_sys;
  double* x;
  double* r;
  double* z;
  double* p;
  double* q;
  const double* f;
  const double* dinv;      // per instance free DOF
  double* slots;
  double* part_pq;         // [n_chunks]
  double* part_rz;         // [2][n_chunks]
  double* part_rr;         // [2][n_chunks]
  double* part_aux;        // [3][n_chunks]: f.f, f.x, |f - Kx|^2
  int32_t* status;         // [n_sys]
  int32_t* iters;          // [n_sys]
  double* tol2;            // [n_sys]
  double* sys_out;         // [n_sys][4]: f.f, f.x, |f-Kx|^2, spare
  int32_t* it_base;        // [1]
  int32_t* n_active;       // [1]
};

enum ElemMode { ELEM_APPLY = 0, ELEM_PCG = 1 };

// y-slots of K applied to the vector `xin` (ELEM_APPLY) or to the PCG search
// direction p = z + beta p formed on the fly (ELEM_PCG), for the tiles of one group.
void launch_elem(const GroupDev& g, int path, const Tile* tiles, const double* E, const double* xin,
                 const PcgDev& s, int mode, int it_k, hipStream_t st);
void launch_sens(const GroupDev& g, const Tile* tiles, const double* dE, const double* x, double* gout,
                 const SysDesc* sys, hipStream_t st);
void launch_diag_elem(const GroupDev& g, const Tile* tiles, const double* E, double* slots, const SysDesc* sys,
                      hipStream_t st);

void launch_simp(const double* rho, double* E, double* dE, int64_t n, double E0, double Emin, double q,
                 hipStream_t st);
void launch_fill(double* a, double v, int64_t n, hipStream_t st);
void launch_fill_i32(int32_t* a, int32_t v, int64_t n, hipStream_t st);
// dinv = 1 / (sum of slots) on the first system of each instance
void launch_dinv(const PcgDev& s, double* dinv, hipStream_t st);
// r = f - (assembled slots if use_slots), z = dinv r, p = 0, partials
void launch_init(const PcgDev& s, int use_slots, hipStream_t st);
void launch_sys_setup(const PcgDev& s, double rtol, hipStream_t st);
void launch_dof1(const PcgDev& s, int it_k, hipStream_t st);
void launch_dof2(const PcgDev& s, int it_k, hipStream_t st);
void launch_advance(const PcgDev& s, int G, hipStream_t st);
// |f - assembled slots|^2 and f.x partials, then per-system sums into sys_out
void launch_residual(const PcgDev& s, hipStream_t st);
// assembled slots -> y in the u layout (zeros elsewhere must be pre-filled);
// diag_mode: only load-0 systems, at their per-instance offset diag_off
void launch_assemble_to_full(const PcgDev& s, const int32_t* free_to_full, double* yfull, int diag_mode,
                             hipStream_t st);
// x (free) <-> u layout
void launch_gather_free(const PcgDev& s, const int32_t* free_to_full, const double* ufull, double* xfree,
                        hipStream_t st);
void launch_scatter_full(const PcgDev& s, const int32_t* free_to_full, const double* xfree, double* ufull,
                         hipStream_t st);
void launch_compliance(const PcgDev& s, double* c, hipStream_t st);

}  // namespace mto
