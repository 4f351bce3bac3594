// Host runtime and C ABI: plan construction (groups, tiles, chunks, device
// buffers), the PCG driver (captured HIP graphs of PCG iterations, polled
// convergence), the true-residual check with restarts, outputs, and autotuning.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mto_internal.hpp"
#include "mto_kernels.hpp"

using namespace mto;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

namespace mto {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
void clear_error() { g_err.clear(); }
}  // namespace mto

namespace {

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? MTO_ENOMEM : MTO_EHIP,                        \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                       \
  } while (0)

constexpr int CHUNK = 1024;  // free DOFs per vector-kernel block (one per thread)
constexpr int N_PROG = 4;    // PCG chunk launches in flight at most

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct GroupHost {
  int p = 0, d = 0, S = 0, ne = 0, nep = 0, mb = 0;
  int n_elems = 0, npad = 0, ncol = 1, waves = 1;
  // LDS-staged contraction (p >= 3): 0 = off, else 64 lds_nc columns per tile, on their own tiles
  int lds_nc = 0, lds_tile_begin = 0, lds_n_tiles = 0;
  // tiles of the first system of each instance (the Schwarz application serves all its systems)
  int ms_tile_begin = 0, ms_n_tiles = 0;
  // per instance: element range [inst_begin[i], inst_begin[i+1]) in the group arrays
  std::vector<int32_t> inst_begin;
  double* kfrag = nullptr;
  double* kfrags = nullptr;  // null without a vector-ALU tail (kfrag serves the LDS-staged kernel then)
  // stored element matrices (mto_set_tile ks = -2): K_e assembled per design, products read them
  int stored = 0;
  double* kst = nullptr;
  double* kfragv = nullptr;
  double* ks = nullptr;
  double* kdiag = nullptr;
  double* kabs = nullptr;
  int32_t* gidx = nullptr;
  int32_t* sidx = nullptr;
  int32_t* msidx = nullptr;
  int32_t* cell = nullptr;
  int tile_begin = 0, n_tiles = 0;
  double flops = 0.0;  // 2 S ne^2 per element column
  std::vector<double> kv;  // host copy of the vertex-block table
  int kv_off = 0;
  // element-block Schwarz smoother: packed inverses [npad/16][ne (ne+1)/2][16], neighbours [8][npad]
  double* binv = nullptr;
  int32_t* nbr = nullptr;
  // QR-error indicator (built at its first use): instance and element of every column,
  // packed order-(p+1) cell tables
  std::vector<int32_t> eid_h, einst_h;
  int32_t *d_eid = nullptr, *d_einst = nullptr;
  double* qtab = nullptr;
};

// Geometric hierarchy of the multigrid preconditioner (levels 1..L).
struct MgHost {
  int L = 0;
  // per level l (index l-1): chunk ranges in the device chunk arrays
  std::vector<int> sys_begin, sys_count, inst_begin, inst_count;
  // per level l: chunks of each instance serving all its systems (sys = its first, nsys = its count)
  std::vector<int> isys_begin, isys_count;
  // whole-grid chunks of the coarsest level (one per system, one per
  // instance) for the dense coarse kernels; the node-parallel kernels use the
  // MG_CHUNK-node chunks above on every level
  int coarse_sys_begin = 0, coarse_inst_begin = 0, coarse_isys_begin = 0;
  std::vector<MgChunk> chunks;  // all levels: system chunks then instance chunks, per level
  MgChunk* d_chunks = nullptr;
  double *A = nullptr, *dinv = nullptr, *mask = nullptr;  // operators [op nodes]
  double *r = nullptr, *e = nullptr, *e2 = nullptr;       // vectors [vec nodes]
  double* dense = nullptr;                                // coarsest inverses
  int32_t* vfree = nullptr;                               // level 1: free index of vertex DOFs
  MgElem* elems = nullptr;
  double* kv = nullptr;
  double* band = nullptr;  // coarsest: band Cholesky factors
  double* scr = nullptr;   // coarsest: inverse in band order (setup scratch)
  int coarse_nmax = 0, coarse_bmax = 0;
  const MgChunk* sysc(int l) const { return d_chunks + sys_begin[l - 1]; }
  const MgChunk* instc(int l) const { return d_chunks + inst_begin[l - 1]; }
  const MgChunk* coarse_sysc() const { return d_chunks + coarse_sys_begin; }
  const MgChunk* coarse_instc() const { return d_chunks + coarse_inst_begin; }
  const MgChunk* isysc(int l) const { return d_chunks + isys_begin[l - 1]; }
  const MgChunk* coarse_isysc() const { return d_chunks + coarse_isys_begin; }
};

struct mto_plan {
  int device = 0;
  mto_params prm{};
  int n_inst = 0, n_sys = 0;
  // per instance
  std::vector<int64_t> cell_off, n_cells, u_off, n_dof, g_off, c_off, n_free, free_off;
  std::vector<int32_t> L;
  int64_t n_cells_tot = 0, n_u = 0, n_g = 0, n_c = 0, n_free_inst_tot = 0, n_vec = 0, n_slots_tot = 0;
  int64_t n_elements = 0;
  std::vector<SysDesc> sys;
  std::vector<Chunk> chunks;
  std::vector<GroupHost> groups;
  std::vector<Tile> tiles;
  std::vector<DevBuf> allocs;
  // device arrays
  SysDesc* d_sys = nullptr;
  Chunk* d_chunks = nullptr;
  Tile* d_tiles = nullptr;
  size_t tiles_cap = 0;
  double *E = nullptr, *dE = nullptr;
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *f = nullptr, *dinv = nullptr;
  double* slots = nullptr;
  double* slots_lo = nullptr;  // low parts of the double-double residual contraction
  double *xs_hi = nullptr, *xs_lo = nullptr;  // refined solution, double-double
  double *part_pq = nullptr, *part_rz = nullptr, *part_rr = nullptr, *part_aux = nullptr, *part_xx = nullptr;
  // per-system results in one block, fetched with one copy: status and
  // iteration count (int32 each, one double's width per system), then
  // sys_out [n_sys][4]
  double* sysblk = nullptr;
  int32_t *status = nullptr, *iters = nullptr, *it_base = nullptr;
  int32_t* bad_rho = nullptr;  // [1]: set by the moduli kernel for an invalid density
  double* progress = nullptr;  // [2], written by each chunk's last kernel
  double *tol2 = nullptr, *sys_out = nullptr;
  int32_t* dd_ok = nullptr;  // [n_sys]
  int32_t* rep_skip = nullptr;  // [n_sys]
  int32_t* rep_count = nullptr;  // [n_sys]
  double* h_sysblk = nullptr;  // host pinned copy of sysblk
  int32_t* f2f = nullptr;
  double* kspr = nullptr;  // ground springs per instance free DOF (NULL: none)
  int64_t *d_inst_cell_off = nullptr, *d_inst_g_off = nullptr;  // [n_inst + 1], [n_inst]
  int32_t *d_inst_c_off = nullptr, *d_inst_L = nullptr;
  // host pinned: one progress report per chunk launch in flight
  double* h_prog = nullptr;  // [N_PROG][2]
  hipEvent_t ev[N_PROG] = {};
  // per-iteration decrease of log(rr / tol2) seen last (0: none yet)
  double rate_hint = 0.0;
  hipStream_t cap_stream = nullptr;
  // the multigrid set-up runs on side_stream beside the Schwarz block inverses
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // graphs
  hipGraphExec_t chunk_exec = nullptr, small_exec = nullptr;
  int chunk_G = 0, small_G = 0;
  // bound (captured) buffers
  bool bound = false;
  const double* b_rho = nullptr;
  double *b_u = nullptr, *b_c = nullptr, *b_g = nullptr;
  hipGraphExec_t setup_exec = nullptr, resid_exec = nullptr, restart_exec = nullptr, out_exec = nullptr;
  MgHost mg;
  // the product of all groups in one launch (k_elem_fused): on when the
  // autotuner measured it faster than one launch per group
  bool fused = false;
  int fused_tile_begin = 0, fused_n_tiles = 0;
  size_t fused_lds = 0;
  GroupDev* d_groups_cur = nullptr;  // the groups' current device views (after the last rebuild_tiles)
  // element-block Schwarz smoother (MTO_PRECOND_MG_ASM)
  GroupDev* d_groups = nullptr;
  int32_t *d_el_group = nullptr, *d_el_col = nullptr;
  double* slots2 = nullptr;  // the Schwarz products, assembled like the slots
  double asm_omega = 0.0;
  // QR-error indicator: per instance first system, load cases, output offset, elements
  bool qr_ready = false, ad_ready = false;
  std::vector<int32_t> inst_nelx, inst_nely;
  GroupDev* d_ad_groups = nullptr;
  int32_t *d_ad_elgroup = nullptr, *d_ad_elcol = nullptr, *d_ad_nelx = nullptr, *d_ad_nely = nullptr;
  int64_t* d_ad_base = nullptr;
  int32_t *d_qr_sys0 = nullptr, *d_qr_L = nullptr, *d_qr_nel = nullptr;
  int64_t* d_qr_eoff = nullptr;

  PcgDev pcg() const {
    PcgDev s{};
    s.sys = d_sys;
    s.chunks = d_chunks;
    s.n_chunks = (int32_t)chunks.size();
    s.n_sys = n_sys;
    s.z_jacobi = prm.precond != MTO_PRECOND_MG_ASM;
    s.x = x;
    s.r = r;
    s.z = z;
    s.p = p;
    s.q = q;
    s.f = f;
    s.dinv = dinv;
    s.kspr = kspr;
    s.slots = slots;
    s.part_pq = part_pq;
    s.part_rz = part_rz;
    s.part_rr = part_rr;
    s.part_xx = part_xx;
    s.part_aux = part_aux;
    s.status = status;
    s.iters = iters;
    s.tol2 = tol2;
    s.sys_out = sys_out;
    s.dd_ok = dd_ok;
    s.rep_skip = rep_skip;
    s.rep_count = rep_count;
    s.it_base = it_base;
    s.progress = progress;
    s.bad_rho = bad_rho;
    return s;
  }
  GroupDev gdev(const GroupHost& g) const {
    GroupDev o{};
    o.p = g.p;
    o.d = g.d;
    o.S = g.S;
    o.npad = g.npad;
    o.n_elems = g.n_elems;
    o.tile_begin = g.tile_begin;
    o.n_tiles = g.n_tiles;
    o.ncol = g.ncol;
    o.waves = g.waves;
    o.xcd_run = n_sys > 1 ? 8 : 0;  // several systems may stop at different iterations
    o.lds_nc = g.lds_nc;
    o.lds_tile_begin = g.lds_tile_begin;
    o.lds_n_tiles = g.lds_n_tiles;
    o.ms_tile_begin = g.ms_tile_begin;
    o.ms_n_tiles = g.ms_n_tiles;
    o.kfrag = g.kfrag;
    o.kfrags = g.kfrags ? g.kfrags : g.kfrag;
    o.kst = g.kst;
    o.stored = g.stored;
    o.kfragv = g.kfragv;
    o.ks = g.ks;
    o.kdiag = g.kdiag;
    o.kabs = g.kabs;
    o.gidx = g.gidx;
    o.sidx = g.sidx;
    o.msidx = g.msidx;
    o.cell = g.cell;
    return o;
  }
};

namespace {

template <class T>
int dev_alloc(mto_plan* P, T** out, size_t count) {
  void* ptr = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) return fail(MTO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  P->allocs.push_back({ptr, bytes});
  *out = (T*)ptr;
  return MTO_OK;
}

template <class T>
int dev_upload(mto_plan* P, T** out, const std::vector<T>& h) {
  int rc = dev_alloc(P, out, h.size());
  if (rc) return rc;
  if (!h.empty()) HIP_TRY(hipMemcpy(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return MTO_OK;
}

void destroy_graphs(mto_plan* P) {
  hipGraphExec_t* gs[] = {&P->chunk_exec, &P->small_exec, &P->setup_exec, &P->resid_exec, &P->restart_exec, &P->out_exec};
  for (auto g : gs)
    if (*g) {
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  P->bound = false;
}

// Tiles for every group with its current ncol, then the tiles of the
// LDS-staged contraction (64 lds_nc columns) for the groups that use it, then
// the tiles of the first system of every instance (16 ncol columns) for the
// Schwarz application; uploads them.
int rebuild_tiles(mto_plan* P) {
  P->tiles.clear();
  for (int pass = 0; pass < 3; ++pass)
  for (size_t gi = 0; gi < P->groups.size(); ++gi) {
    GroupHost& g = P->groups[gi];
    if (P->prm.kernel_path == MTO_PATH_PLAIN) {
      g.ncol = 4;  // one 64-thread block per 64-column tile
      g.lds_nc = 0;
    }
    if (pass == 1 && g.lds_nc == 0) {
      g.lds_tile_begin = (int)P->tiles.size();
      g.lds_n_tiles = 0;
      continue;
    }
    const int tile_cols = pass == 1 ? 64 * g.lds_nc : pass == 2 ? asm_cols_of(g.p) : 16 * g.ncol;
    (pass == 0 ? g.tile_begin : pass == 1 ? g.lds_tile_begin : g.ms_tile_begin) = (int)P->tiles.size();
    for (int i = 0; i < P->n_inst; ++i) {
      const int a = g.inst_begin[i], b = g.inst_begin[i + 1];
      if (a == b) continue;
      for (int l = 0; l < (pass == 2 ? 1 : P->L[i]); ++l) {
        int sysi = 0;
        for (int k = 0; k < i; ++k) sysi += P->L[k];
        sysi += l;
        const SysDesc& sd = P->sys[sysi];
        for (int e = a; e < b; e += tile_cols) {
          Tile t{};
          t.dof_off = sd.dof_off;
          t.slot_off = sd.slot_off;
          t.group = (int32_t)gi;
          t.sys = sysi;
          t.elem_begin = e;
          t.count = std::min(tile_cols, b - e);
          t.pc_begin = pass == 2 ? P->L[i] : sd.chunk_begin;  // Schwarz tiles: the instance's system count
          t.pc_end = sd.chunk_end;
          P->tiles.push_back(t);
        }
      }
    }
    if (pass == 0)
      g.n_tiles = (int)P->tiles.size() - g.tile_begin;
    else if (pass == 1)
      g.lds_n_tiles = (int)P->tiles.size() - g.lds_tile_begin;
    else
      g.ms_n_tiles = (int)P->tiles.size() - g.ms_tile_begin;
  }
  // the combined tiles of the fused product: 64 columns, groups by decreasing work per column
  {
    std::vector<int> order(P->groups.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      const GroupHost &a = P->groups[x], &b = P->groups[y];
      return (double)a.S * a.ne * a.ne > (double)b.S * b.ne * b.ne;
    });
    P->fused_tile_begin = (int)P->tiles.size();
    P->fused_lds = 0;
    for (int gi : order) {
      const GroupHost& g = P->groups[gi];
      P->fused_lds = std::max(P->fused_lds, elem_lds_staged_bytes(g.p, 1));
      for (int i = 0; i < P->n_inst; ++i) {
        const int a = g.inst_begin[i], b = g.inst_begin[i + 1];
        if (a == b) continue;
        int sysi = 0;
        for (int k = 0; k < i; ++k) sysi += P->L[k];
        for (int l = 0; l < P->L[i]; ++l) {
          const SysDesc& sd = P->sys[sysi + l];
          for (int e = a; e < b; e += 64) {
            Tile t{};
            t.dof_off = sd.dof_off;
            t.slot_off = sd.slot_off;
            t.group = (int32_t)gi;
            t.sys = sysi + l;
            t.elem_begin = e;
            t.count = std::min(64, b - e);
            t.pc_begin = sd.chunk_begin;
            t.pc_end = sd.chunk_end;
            P->tiles.push_back(t);
          }
        }
      }
    }
    P->fused_n_tiles = (int)P->tiles.size() - P->fused_tile_begin;
  }
  if (P->tiles.size() > P->tiles_cap) {
    if (P->d_tiles) {
      (void)hipFree(P->d_tiles);
      for (auto& a : P->allocs)
        if (a.ptr == P->d_tiles) a.ptr = nullptr;
    }
    int rc = dev_alloc(P, &P->d_tiles, P->tiles.size());
    if (rc) return rc;
    P->tiles_cap = P->tiles.size();
  }
  if (!P->tiles.empty())
    HIP_TRY(hipMemcpy(P->d_tiles, P->tiles.data(), P->tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
  {
    std::vector<GroupDev> gd;
    for (auto& g : P->groups) gd.push_back(P->gdev(g));
    if (!P->d_groups_cur) {
      int rc = dev_alloc(P, &P->d_groups_cur, gd.size());
      if (rc) return rc;
    }
    if (!gd.empty()) HIP_TRY(hipMemcpy(P->d_groups_cur, gd.data(), gd.size() * sizeof(GroupDev), hipMemcpyHostToDevice));
  }
  destroy_graphs(P);
  return MTO_OK;
}

// ---- autotune cache: one text line per (arch, p, d, size class) ----
// "arch p d size_class ncol ks us"; size class = floor(log2(element columns
// of the group)), since the best tile shape of a group of a few elements and
// of a full mesh differ.
struct TileKey {
  std::string arch;
  int p, d, size_class;
  bool operator<(const TileKey& o) const {
    if (arch != o.arch) return arch < o.arch;
    if (p != o.p) return p < o.p;
    if (d != o.d) return d < o.d;
    return size_class < o.size_class;
  }
};
struct TileChoice {
  int ncol, ks;
  double us;
};

int size_class(double columns) {
  int c = 0;
  while (columns >= 2.0 && c < 40) {
    columns *= 0.5;
    ++c;
  }
  return c;
}

// Reads the cache if the file exists (a missing file is an empty cache);
// false on a malformed line.
bool read_tile_cache(const char* path, std::map<TileKey, TileChoice>& out) {
  FILE* fh = fopen(path, "r");
  if (!fh) return true;
  char line[1024];
  bool ok = true;
  while (fgets(line, sizeof line, fh)) {
    if (!std::strchr(line, '\n') && !feof(fh)) {  // longer than the buffer: a comment may be, an entry not
      const bool comment = line[0] == '#';
      int ch;
      while ((ch = fgetc(fh)) != EOF && ch != '\n') {
      }
      if (comment) continue;
      ok = false;
      break;
    }
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[64];
    TileKey k;
    TileChoice v;
    if (sscanf(line, "%63s %d %d %d %d %d %lf", arch, &k.p, &k.d, &k.size_class, &v.ncol, &v.ks, &v.us) != 7 ||
        (v.ncol != 1 && v.ncol != 2 && v.ncol != 4) || v.ks < -2 || v.ks == -1 || v.ks > 8 || k.p < 0 ||
        k.p > MTO_MAX_P || (v.ks == -2 && (k.p == 0 || v.ncol != 1)) ||
        k.d < 0 || k.d > MTO_MAX_D * MTO_MAX_P || (k.p > 0 && k.d < 1) || (k.p > 0 && k.d > MTO_MAX_D) ||
        (k.p > 0 && v.ks == 0 && (k.p < 3 || v.ncol == 4)) || (k.p == 0 && (v.ks != 0 || v.ncol == 4))) {
      ok = false;
      break;
    }
    k.arch = arch;
    out[k] = v;
  }
  fclose(fh);
  return ok;
}

bool write_tile_cache(const char* path, const std::map<TileKey, TileChoice>& c) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fh = fopen(tmp.c_str(), "w");
  if (!fh) return false;
  fprintf(fh, "# element-contraction tile shapes: arch p d size_class(log2 columns) ncol ks us_per_launch\n"
              "# ks 0: LDS-staged tables, 64 ncol columns per tile; ks -2: stored element matrices\n"
              "# p 0: the plan's choice between one launch for all its d groups (ncol 1) and one per group (ncol 2)\n");
  for (auto& kv : c)
    fprintf(fh, "%s %d %d %d %d %d %.3f\n", kv.first.arch.c_str(), kv.first.p, kv.first.d, kv.first.size_class,
            kv.second.ncol, kv.second.ks, kv.second.us);
  const bool ok = fclose(fh) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MTO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return MTO_OK;
}

// Builds the multigrid hierarchy: per instance the vertex grid of the mesh
// (level 1) and its coarsenings by two, until the largest instance's grid
// has at most mg_coarse_max DOFs (smaller instances continue to coarsen,
// down to one element, so every instance has the same number of levels).
int build_mg(mto_plan* P, const std::vector<InstanceHost>& I) {
  MgHost& M = P->mg;
  const int n = P->n_inst;
  std::vector<std::vector<std::pair<int, int>>> dims(n);
  const int64_t cmax = P->prm.mg_coarse_max;
  int L = 1;
  for (int i = 0; i < n; ++i) {
    int nx = I[i].nelx, ny = I[i].nely, l = 1;
    while ((2LL * (nx + 1) * (ny + 1) > cmax || 2 * std::min(nx, ny) + 5 > MG_BAND_MAX) &&
           (nx > 1 || ny > 1)) {
      nx = (nx + 1) / 2;
      ny = (ny + 1) / 2;
      ++l;
    }
    L = std::max(L, l);
  }
  for (int i = 0; i < n; ++i) {
    int nx = I[i].nelx, ny = I[i].nely;
    for (int l = 1; l <= L; ++l) {
      dims[i].emplace_back(nx, ny);
      nx = (nx + 1) / 2;
      ny = (ny + 1) / 2;
    }
  }
  M.L = L;
  // operator node offsets [l][instance], vector node offsets [l][system]
  std::vector<std::vector<int64_t>> op(L, std::vector<int64_t>(n)), vec(L, std::vector<int64_t>(P->n_sys));
  int64_t op_tot = 0, vec_tot = 0, dense_tot = 0, band_tot = 0;
  std::vector<int64_t> dense_off(n), band_off(n);
  for (int l = 0; l < L; ++l)
    for (int i = 0; i < n; ++i) {
      op[l][i] = op_tot;
      op_tot += (int64_t)(dims[i][l].first + 1) * (dims[i][l].second + 1);
    }
  for (int l = 0; l < L; ++l)
    for (int s = 0; s < P->n_sys; ++s) {
      const int i = P->sys[s].inst;
      vec[l][s] = vec_tot;
      vec_tot += (int64_t)(dims[i][l].first + 1) * (dims[i][l].second + 1);
    }
  for (int i = 0; i < n; ++i) {
    const int64_t N = (int64_t)(dims[i][L - 1].first + 1) * (dims[i][L - 1].second + 1);
    const int bw = 2 * std::min(dims[i][L - 1].first, dims[i][L - 1].second) + 5;  // band width, as in the kernels
    if (2 * N > MG_COARSE_MAX || bw > MG_BAND_MAX) return fail(MTO_EINVAL, "multigrid: coarsest grid too large");
    dense_off[i] = dense_tot;
    dense_tot += 4 * N * N;
    band_off[i] = band_tot;
    band_tot += mg_band_doubles(2 * N);
    M.coarse_nmax = std::max<int>(M.coarse_nmax, (int)(2 * N));
    M.coarse_bmax = std::max(M.coarse_bmax, bw);
  }
  // element table per instance for the level-1 assembly
  std::vector<int64_t> elem_off(n);
  std::vector<MgElem> elems;
  std::map<std::pair<int, int>, int> gidx;
  std::vector<double> kvpool;
  for (size_t g = 0; g < P->groups.size(); ++g) {
    gidx[{P->groups[g].p, P->groups[g].d}] = (int)g;
    P->groups[g].kv_off = (int)kvpool.size();
    kvpool.insert(kvpool.end(), P->groups[g].kv.begin(), P->groups[g].kv.end());
  }
  for (int i = 0; i < n; ++i) {
    elem_off[i] = (int64_t)elems.size();
    for (size_t e = 0; e < I[i].p.size(); ++e) {
      const GroupHost& G = P->groups[gidx[{(int)I[i].p[e], (int)I[i].d[e]}]];
      elems.push_back(MgElem{(int32_t)(P->cell_off[i] + I[i].cell_off[e]), G.kv_off, G.S, 0});
    }
  }
  // level-1 free index of each vertex DOF (vertex DOFs are the first 2 N1 of the numbering)
  std::vector<int32_t> vfree;
  int64_t n1_tot = 0;
  for (int i = 0; i < n; ++i) n1_tot += (int64_t)(I[i].nelx + 1) * (I[i].nely + 1);
  vfree.assign(2 * (size_t)n1_tot, -1);
  for (int i = 0; i < n; ++i) {
    const int64_t N1 = (int64_t)(I[i].nelx + 1) * (I[i].nely + 1);
    for (int64_t k = 0; k < 2 * N1; ++k) vfree[2 * op[0][i] + k] = I[i].full_to_free[k];
  }
  // chunks: per level the system chunks, then the instance chunks
  M.sys_begin.assign(L, 0);
  M.sys_count.assign(L, 0);
  M.inst_begin.assign(L, 0);
  M.inst_count.assign(L, 0);
  M.isys_begin.assign(L, 0);
  M.isys_count.assign(L, 0);
  std::vector<int> first_sys(n, -1);
  for (int s = P->n_sys - 1; s >= 0; --s) first_sys[P->sys[s].inst] = s;
  auto make = [&](int l, int i, int sys, int nb, int ne, int nsys = 1) {
    MgChunk c{};
    c.sys = sys;
    c.nsys = nsys;
    c.inst = i;
    c.level = l + 1;
    c.node_begin = nb;
    c.node_end = ne;
    c.nx = dims[i][l].first;
    c.ny = dims[i][l].second;
    c.op = op[l][i];
    c.vec = sys >= 0 ? vec[l][sys] : -1;
    if (l > 0) {
      c.fnx = dims[i][l - 1].first;
      c.fny = dims[i][l - 1].second;
      c.fop = op[l - 1][i];
      c.fvec = sys >= 0 ? vec[l - 1][sys] : -1;
    } else {
      c.fop = c.fvec = -1;
    }
    if (l + 1 < L) {
      c.cnx = dims[i][l + 1].first;
      c.cny = dims[i][l + 1].second;
      c.cop = op[l + 1][i];
      c.cvec = sys >= 0 ? vec[l + 1][sys] : -1;
    } else {
      c.cop = c.cvec = -1;
    }
    c.dense_off = dense_off[i];
    c.band_off = band_off[i];
    c.elem_off = elem_off[i];
    if (sys >= 0) {
      c.dof_off = P->sys[sys].dof_off;
      c.slot_off = P->sys[sys].slot_off;
      c.nfv = P->sys[sys].nfv;
      c.nfe = P->sys[sys].nfe;
    }
    return c;
  };
  for (int l = 0; l < L; ++l) {
    M.sys_begin[l] = (int)M.chunks.size();
    for (int s = 0; s < P->n_sys; ++s) {
      const int i = P->sys[s].inst;
      const int N = (dims[i][l].first + 1) * (dims[i][l].second + 1);
      for (int b = 0; b < N; b += MG_CHUNK) M.chunks.push_back(make(l, i, s, b, std::min(N, b + MG_CHUNK)));
    }
    M.sys_count[l] = (int)M.chunks.size() - M.sys_begin[l];
    M.inst_begin[l] = (int)M.chunks.size();
    for (int i = 0; i < n; ++i) {
      const int N = (dims[i][l].first + 1) * (dims[i][l].second + 1);
      for (int b = 0; b < N; b += MG_CHUNK) M.chunks.push_back(make(l, i, -1, b, std::min(N, b + MG_CHUNK)));
    }
    M.inst_count[l] = (int)M.chunks.size() - M.inst_begin[l];
    M.isys_begin[l] = (int)M.chunks.size();
    for (int i = 0; i < n; ++i) {
      const int N = (dims[i][l].first + 1) * (dims[i][l].second + 1);
      for (int b = 0; b < N; b += MG_CHUNK)
        M.chunks.push_back(make(l, i, first_sys[i], b, std::min(N, b + MG_CHUNK), P->L[i]));
    }
    M.isys_count[l] = (int)M.chunks.size() - M.isys_begin[l];
  }
  M.coarse_sys_begin = (int)M.chunks.size();
  for (int s = 0; s < P->n_sys; ++s) {
    const int i = P->sys[s].inst;
    M.chunks.push_back(make(L - 1, i, s, 0, (dims[i][L - 1].first + 1) * (dims[i][L - 1].second + 1)));
  }
  M.coarse_inst_begin = (int)M.chunks.size();
  for (int i = 0; i < n; ++i)
    M.chunks.push_back(make(L - 1, i, -1, 0, (dims[i][L - 1].first + 1) * (dims[i][L - 1].second + 1)));
  M.coarse_isys_begin = (int)M.chunks.size();
  for (int i = 0; i < n; ++i)
    M.chunks.push_back(
        make(L - 1, i, first_sys[i], 0, (dims[i][L - 1].first + 1) * (dims[i][L - 1].second + 1), P->L[i]));
  int rc;
  if ((rc = dev_upload(P, &M.d_chunks, M.chunks)) || (rc = dev_alloc(P, &M.A, 36 * (size_t)op_tot)) ||
      (rc = dev_alloc(P, &M.dinv, 2 * (size_t)op_tot)) || (rc = dev_alloc(P, &M.mask, 2 * (size_t)op_tot)) ||
      (rc = dev_alloc(P, &M.r, 2 * (size_t)vec_tot)) || (rc = dev_alloc(P, &M.e, 2 * (size_t)vec_tot)) ||
      (rc = dev_alloc(P, &M.e2, 2 * (size_t)vec_tot)) ||
      (rc = dev_alloc(P, &M.dense, (size_t)dense_tot)) || (rc = dev_alloc(P, &M.band, (size_t)band_tot)) ||
      (rc = dev_alloc(P, &M.scr, (size_t)dense_tot)) ||
      (rc = dev_upload(P, &M.vfree, vfree)) || (rc = dev_upload(P, &M.elems, elems)) ||
      (rc = dev_upload(P, &M.kv, kvpool)))
    return rc;
  launch_fill(M.band, 0.0, band_tot, 0);  // the factor kernels write only inside the band
  launch_fill(M.e, 0.0, 2 * vec_tot, 0);
  launch_fill(M.e2, 0.0, 2 * vec_tot, 0);
  launch_fill(M.r, 0.0, 2 * vec_tot, 0);
  return check_launch("multigrid setup");
}

// Tables of the element-block Schwarz smoother: the group and column of every
// element of every instance, each column's eight neighbours, and the block
// inverses (filled per design by the setup).
int build_asm(mto_plan* P, const std::vector<InstanceHost>& I) {
  const int n = P->n_inst;
  std::vector<int64_t> base(n + 1, 0);
  for (int i = 0; i < n; ++i) base[i + 1] = base[i] + (int64_t)I[i].nelx * I[i].nely;
  std::vector<int32_t> el_group(base[n], -1), el_col(base[n], -1);
  std::map<std::pair<int, int>, int> gid;
  for (size_t g = 0; g < P->groups.size(); ++g) gid[{P->groups[g].p, P->groups[g].d}] = (int)g;
  std::vector<int> next(P->groups.size(), 0);
  for (int i = 0; i < n; ++i)
    for (size_t e = 0; e < I[i].p.size(); ++e) {
      const int g = gid[{(int)I[i].p[e], (int)I[i].d[e]}];
      el_group[base[i] + e] = g;
      el_col[base[i] + e] = next[g]++;  // group columns: instance order, then element order
    }
  std::vector<GroupDev> gd;
  int rc;
  for (size_t g = 0; g < P->groups.size(); ++g) {
    GroupHost& G = P->groups[g];
    std::vector<int32_t> nbr(8 * (size_t)G.npad, -1);
    for (int i = 0; i < n; ++i) {
      const int nx = I[i].nelx, ny = I[i].nely;
      for (int e = 0; e < nx * ny; ++e) {
        if (el_group[base[i] + e] != (int)g) continue;
        const int k = el_col[base[i] + e], ex = e % nx, ey = e / nx;
        int m = 0;
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy) continue;
            const int x = ex + dx, y = ey + dy;
            if (x >= 0 && x < nx && y >= 0 && y < ny) nbr[(size_t)m * G.npad + k] = (int32_t)(base[i] + y * nx + x);
            ++m;
          }
      }
    }
    if ((int64_t)G.ne * (G.ne + 1) / 2 * G.npad >= ((int64_t)1 << 31))
      return fail(MTO_EINVAL, "Schwarz smoother: too many elements of one (p, d) group for 32-bit block offsets");
    if ((rc = dev_upload(P, &G.nbr, nbr)) || (rc = dev_alloc(P, &G.binv, (size_t)asm_ntp_of(G.p) * G.npad))) return rc;
    gd.push_back(P->gdev(G));
  }
  if ((rc = dev_upload(P, &P->d_groups, gd)) || (rc = dev_upload(P, &P->d_el_group, el_group)) ||
      (rc = dev_upload(P, &P->d_el_col, el_col)) || (rc = dev_alloc(P, &P->slots2, P->n_slots_tot)))
    return rc;
  launch_fill(P->slots2, 0.0, P->n_slots_tot, 0);  // slots no element writes read as zero
  P->asm_omega = P->prm.mg_omega > 0.0 ? P->prm.mg_omega : 2.0 / (9.0 * 1.05);
  return MTO_OK;
}

int build_plan(const mto_problem* probs, int n, const mto_params* prm, mto_plan** out) {
  if (!out) return fail(MTO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || n < 1 || !prm) return fail(MTO_EINVAL, "no problems or params");
  if (!(prm->rtol > 0.0) || !(prm->E0 > 0.0) || !(prm->Emin >= 0.0) || !(prm->Emin <= prm->E0) ||
      !(prm->nu > -1.0 && prm->nu < 0.5) || !(prm->q >= 1.0))
    return fail(MTO_EINVAL, "params out of range (rtol > 0, 0 <= Emin <= E0, -1 < nu < 0.5, q >= 1)");
  if (prm->kernel_path != MTO_PATH_MFMA && prm->kernel_path != MTO_PATH_PLAIN)
    return fail(MTO_EINVAL, "unknown kernel_path");
  if (prm->precond != MTO_PRECOND_JACOBI && prm->precond != MTO_PRECOND_MG && prm->precond != MTO_PRECOND_MG_ASM)
    return fail(MTO_EINVAL, "unknown precond");
  if (prm->stored_matrices != 0 && prm->stored_matrices != 1) return fail(MTO_EINVAL, "stored_matrices must be 0 or 1");
  if (prm->precond == MTO_PRECOND_MG_ASM && !(prm->mg_omega < 2.0 / 9.0))
    return fail(MTO_EINVAL, "Schwarz smoother weight must be below 2/9 (<= 0 selects the default)");
  std::vector<InstanceHost> I(n);
  for (int i = 0; i < n; ++i) {
    std::string err;
    int rc = build_instance(probs[i], I[i], err);
    if (rc) return fail(rc, "instance " + std::to_string(i) + ": " + err);
  }
  mto_plan* P = new mto_plan();
  P->prm = *prm;
  // Default chunk of captured iterations: Jacobi runs thousands of short
  // iterations, the multigrid tens of long ones (a stopped system still
  // launches the rest of its chunk, which then returns at once).
  if (P->prm.iters_per_launch <= 0) P->prm.iters_per_launch = P->prm.precond == MTO_PRECOND_JACOBI ? 32 : 8;
  if (P->prm.iters_per_launch % 2) P->prm.iters_per_launch += 1;  // keeps the parity of it_base even
  if (P->prm.max_restarts < 0) P->prm.max_restarts = 3;
  if (P->prm.mg_coarse_max <= 0 || P->prm.mg_coarse_max > MG_COARSE_MAX) P->prm.mg_coarse_max = MG_COARSE_MAX;
  (void)hipGetDevice(&P->device);
  P->n_inst = n;
  auto cleanup = [&](int rc) {
    mto_plan_destroy(P);
    return rc;
  };

  // instance offsets and systems
  P->cell_off.resize(n);
  P->n_cells.resize(n);
  P->u_off.resize(n);
  P->n_dof.resize(n);
  P->g_off.resize(n);
  P->c_off.resize(n);
  P->n_free.resize(n);
  P->free_off.resize(n);
  P->L.resize(n);
  int64_t slot_acc = 0, vec_acc = 0, diag_acc = 0;
  for (int i = 0; i < n; ++i) {
    P->cell_off[i] = P->n_cells_tot;
    P->n_cells[i] = I[i].n_cells;
    P->u_off[i] = P->n_u;
    P->n_dof[i] = I[i].n_dof;
    P->g_off[i] = P->n_g;
    P->c_off[i] = P->n_c;
    P->n_free[i] = I[i].n_free;
    P->free_off[i] = P->n_free_inst_tot;
    P->L[i] = I[i].L;
    P->inst_nelx.push_back(I[i].nelx);
    P->inst_nely.push_back(I[i].nely);
    P->n_cells_tot += I[i].n_cells;
    P->n_u += (int64_t)I[i].L * I[i].n_dof;
    P->n_g += (int64_t)I[i].L * I[i].n_cells;
    P->n_c += I[i].L;
    P->n_free_inst_tot += I[i].n_free;
    P->n_elements += (int64_t)I[i].nelx * I[i].nely;
    for (int l = 0; l < I[i].L; ++l) {
      SysDesc sd{};
      sd.dof_off = vec_acc;
      sd.slot_off = slot_acc;
      sd.u_off = P->u_off[i] + (int64_t)l * I[i].n_dof;
      sd.g_off = P->g_off[i] + (int64_t)l * I[i].n_cells - P->cell_off[i];
      sd.inst_free_off = P->free_off[i];
      sd.diag_off = diag_acc;
      sd.n_free = I[i].n_free;
      sd.nfv = I[i].nfv;
      sd.nfe = I[i].nfe;
      sd.inst = i;
      sd.load = l;
      sd.c_index = (int32_t)(P->c_off[i] + l);
      sd.chunk_begin = (int32_t)P->chunks.size();
      for (int b = 0; b < I[i].n_free; b += CHUNK) {
        Chunk ch{};
        ch.dof_off = sd.dof_off;
        ch.slot_off = sd.slot_off;
        ch.inst_free_off = sd.inst_free_off;
        ch.sys = (int32_t)P->sys.size();
        ch.begin = b;
        ch.end = std::min(I[i].n_free, b + CHUNK);
        ch.nfv = sd.nfv;
        ch.nfe = sd.nfe;
        ch.load = l;
        P->chunks.push_back(ch);
      }
      sd.chunk_end = (int32_t)P->chunks.size();
      for (int k = sd.chunk_begin; k < sd.chunk_end; ++k) {
        P->chunks[k].pc_begin = sd.chunk_begin;
        P->chunks[k].pc_end = sd.chunk_end;
      }
      P->sys.push_back(sd);
      vec_acc += I[i].n_free;
      slot_acc += I[i].n_slots;
    }
    diag_acc += I[i].n_dof;
  }
  P->n_sys = (int)P->sys.size();
  P->n_vec = vec_acc;
  P->n_slots_tot = slot_acc;
  if (P->n_cells_tot >= ((int64_t)1 << 31) || vec_acc >= ((int64_t)1 << 31))
    return cleanup(fail(MTO_EINVAL, "plan too large for 32-bit cell or DOF indices"));

  // groups by (p, d), elements in instance order then element order
  std::map<std::pair<int, int>, int> gid;
  for (int i = 0; i < n; ++i)
    for (size_t e = 0; e < I[i].p.size(); ++e) {
      auto key = std::make_pair((int)I[i].p[e], (int)I[i].d[e]);
      if (!gid.count(key)) {
        int k = (int)gid.size();
        gid[key] = k;
      }
    }
  P->groups.resize(gid.size());
  for (auto& kv : gid) {
    GroupHost& g = P->groups[kv.second];
    g.p = kv.first.first;
    g.d = kv.first.second;
    g.S = g.d * g.d;
    g.ne = ne_of(g.p);
    g.nep = nep_of(g.p);
    g.mb = mb_of(g.p);
    g.ncol = 1;
    g.waves = std::min(4, g.S);
  }
  // order groups by (p, d) for stable output
  for (int gi = 0; gi < (int)P->groups.size(); ++gi) {
    GroupHost& g = P->groups[gi];
    std::vector<std::pair<int, int>> elems;  // (instance, element)
    g.inst_begin.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      g.inst_begin[i] = (int32_t)elems.size();
      for (size_t e = 0; e < I[i].p.size(); ++e)
        if (I[i].p[e] == g.p && I[i].d[e] == g.d) elems.emplace_back(i, (int)e);
    }
    g.inst_begin[n] = (int32_t)elems.size();
    g.n_elems = (int)elems.size();
    g.eid_h.resize(elems.size());
    g.einst_h.resize(elems.size());
    for (size_t k = 0; k < elems.size(); ++k) {
      g.einst_h[k] = elems[k].first;
      g.eid_h[k] = elems[k].second;
    }
    g.npad = std::max(64, (g.n_elems + 63) / 64 * 64);
    std::vector<int32_t> gidx((size_t)g.nep * g.npad, -1), sidx((size_t)g.ne * g.npad, -1), cell(g.npad, 0);
    std::vector<int32_t> msidx((size_t)2 * g.ne * g.npad, -1);
    for (int k = 0; k < g.n_elems; ++k) {
      const int i = elems[k].first, e = elems[k].second;
      const int64_t o = I[i].elem_dof_off[e];
      for (int j = 0; j < g.ne; ++j) {
        gidx[(size_t)j * g.npad + k] = I[i].elem_free[o + j];
        sidx[(size_t)j * g.npad + k] = I[i].elem_slot[o + j];
        msidx[2 * ((size_t)k * g.ne + j)] = I[i].elem_free[o + j];
        msidx[2 * ((size_t)k * g.ne + j) + 1] = I[i].elem_slot[o + j];
      }
      cell[k] = (int32_t)(P->cell_off[i] + I[i].cell_off[e]);
    }
    std::vector<double> ks = subcell_tables(g.p, g.d, P->prm.nu);
    std::vector<double> kfr = mfma_fragments(ks, g.p, g.d);
    std::vector<double> kfv = vertex_fragments(ks, g.p, g.d);
    std::vector<double> kdiag((size_t)g.S * g.ne), kabs((size_t)g.S * g.ne, 0.0);
    for (int s = 0; s < g.S; ++s)
      for (int j = 0; j < g.ne; ++j) {
        kdiag[(size_t)s * g.ne + j] = ks[(size_t)s * g.ne * g.ne + j * g.ne + j];
        for (int k = 0; k < g.ne; ++k) kabs[(size_t)s * g.ne + j] += std::fabs(ks[(size_t)s * g.ne * g.ne + j * g.ne + k]);
      }
    // vertex-vertex blocks [S][corner a0][corner a1][c0][c1] for the level-1 operator
    g.kv.assign((size_t)g.S * 64, 0.0);
    for (int s = 0; s < g.S; ++s)
      for (int a0 = 0; a0 < 4; ++a0)
        for (int a1 = 0; a1 < 4; ++a1)
          for (int c0 = 0; c0 < 2; ++c0)
            for (int c1 = 0; c1 < 2; ++c1) {
              const int l0 = (a0 >> 1) * (g.p + 1) + (a0 & 1), l1 = (a1 >> 1) * (g.p + 1) + (a1 & 1);
              g.kv[(((size_t)s * 4 + a0) * 4 + a1) * 4 + c0 * 2 + c1] =
                  ks[(size_t)s * g.ne * g.ne + (2 * l0 + c0) * g.ne + 2 * l1 + c1];
            }
    int rc;
    if ((rc = dev_upload(P, &g.gidx, gidx)) || (rc = dev_upload(P, &g.sidx, sidx)) ||
        (rc = dev_upload(P, &g.msidx, msidx)) ||
        (rc = dev_upload(P, &g.cell, cell)) || (rc = dev_upload(P, &g.ks, ks)) || (rc = dev_upload(P, &g.kfrag, kfr)) ||
        (rc = dev_upload(P, &g.kfragv, kfv)) ||
        (valu_tail(g.p) && (rc = dev_upload(P, &g.kfrags, staged_fragments(ks, g.p, g.d)))) ||
        (rc = dev_upload(P, &g.kdiag, kdiag)) || (rc = dev_upload(P, &g.kabs, kabs)))
      return cleanup(rc);
    double per_col = 2.0 * g.S * g.ne * g.ne;
    int64_t cols = 0;
    for (int i = 0; i < n; ++i) cols += (int64_t)(g.inst_begin[i + 1] - g.inst_begin[i]) * P->L[i];
    g.flops = per_col * (double)cols;
  }

  // vectors and state
  std::vector<double> fh(P->n_vec, 0.0);
  std::vector<int32_t> f2f(P->n_free_inst_tot);
  for (int s = 0; s < P->n_sys; ++s) {
    const SysDesc& sd = P->sys[s];
    const InstanceHost& Ii = I[sd.inst];
    std::copy(Ii.f.begin() + (size_t)sd.load * Ii.n_free, Ii.f.begin() + (size_t)(sd.load + 1) * Ii.n_free,
              fh.begin() + sd.dof_off);
  }
  for (int i = 0; i < n; ++i) std::copy(I[i].free_to_full.begin(), I[i].free_to_full.end(), f2f.begin() + P->free_off[i]);
  const size_t nch = P->chunks.size();
  int rc;
  if ((rc = dev_upload(P, &P->d_sys, P->sys)) || (rc = dev_upload(P, &P->d_chunks, P->chunks)) ||
      (rc = dev_alloc(P, &P->E, P->n_cells_tot)) || (rc = dev_alloc(P, &P->dE, P->n_cells_tot)) ||
      (rc = dev_alloc(P, &P->x, P->n_vec)) || (rc = dev_alloc(P, &P->r, P->n_vec)) ||
      (rc = dev_alloc(P, &P->z, P->n_vec)) || (rc = dev_alloc(P, &P->p, P->n_vec)) ||
      (rc = dev_alloc(P, &P->q, P->n_vec)) || (rc = dev_upload(P, &P->f, fh)) ||
      (rc = dev_alloc(P, &P->dinv, P->n_free_inst_tot)) || (rc = dev_alloc(P, &P->slots, P->n_slots_tot)) ||
      (rc = dev_alloc(P, &P->slots_lo, P->n_slots_tot)) || (rc = dev_alloc(P, &P->xs_hi, P->n_vec)) ||
      (rc = dev_alloc(P, &P->xs_lo, P->n_vec)) ||
      (rc = dev_alloc(P, &P->part_pq, nch)) || (rc = dev_alloc(P, &P->part_rz, 2 * nch)) ||
      (rc = dev_alloc(P, &P->part_rr, 2 * nch)) || (rc = dev_alloc(P, &P->part_aux, 3 * nch)) ||
      (rc = dev_alloc(P, &P->part_xx, 2 * nch)) ||
      (rc = dev_alloc(P, &P->sysblk, 5 * (size_t)P->n_sys)) ||
      (rc = dev_alloc(P, &P->it_base, 1)) || (rc = dev_alloc(P, &P->progress, 2)) ||
      (rc = dev_alloc(P, &P->bad_rho, 1)) ||
      (rc = dev_alloc(P, &P->tol2, P->n_sys)) || (rc = dev_alloc(P, &P->dd_ok, P->n_sys)) ||
      (rc = dev_alloc(P, &P->rep_skip, P->n_sys)) || (rc = dev_alloc(P, &P->rep_count, P->n_sys)) ||
      (rc = dev_upload(P, &P->f2f, f2f)))
    return cleanup(rc);
  P->status = reinterpret_cast<int32_t*>(P->sysblk);
  P->iters = P->status + P->n_sys;
  P->sys_out = P->sysblk + P->n_sys;
  if (hipHostMalloc((void**)&P->h_sysblk, 5 * (size_t)P->n_sys * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(MTO_ENOMEM, "hipHostMalloc failed"));
  {
    bool any = false;
    for (int i = 0; i < n; ++i) any |= !I[i].springs.empty();
    if (any) {
      std::vector<double> ks(P->n_free_inst_tot, 0.0);
      for (int i = 0; i < n; ++i)
        for (auto& sp : I[i].springs) ks[P->free_off[i] + sp.first] += sp.second;
      if ((rc = dev_upload(P, &P->kspr, ks))) return cleanup(rc);
    }
  }
  {
    std::vector<int64_t> co(P->cell_off), go(P->g_off);
    co.push_back(P->n_cells_tot);
    std::vector<int32_t> cc(n), ll(P->L);
    for (int i = 0; i < n; ++i) cc[i] = (int32_t)P->c_off[i];
    if ((rc = dev_upload(P, &P->d_inst_cell_off, co)) || (rc = dev_upload(P, &P->d_inst_g_off, go)) ||
        (rc = dev_upload(P, &P->d_inst_c_off, cc)) || (rc = dev_upload(P, &P->d_inst_L, ll)))
      return cleanup(rc);
  }
  // slots that no element writes (missing neighbours) must read as zero forever
  launch_fill(P->slots, 0.0, P->n_slots_tot, 0);
  launch_fill(P->slots_lo, 0.0, P->n_slots_tot, 0);
  launch_fill(P->x, 0.0, P->n_vec, 0);
  launch_fill_i32(P->dd_ok, 0, P->n_sys, 0);
  launch_fill_i32(P->rep_skip, 1, P->n_sys, 0);
  launch_fill_i32(P->rep_count, 0, P->n_sys, 0);
  if ((rc = check_launch("fill"))) return cleanup(rc);
  if (hipHostMalloc((void**)&P->h_prog, 2 * N_PROG * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(MTO_ENOMEM, "hipHostMalloc failed"));
  for (int k = 0; k < N_PROG; ++k)
    if (hipEventCreateWithFlags(&P->ev[k], hipEventDisableTiming) != hipSuccess)
      return cleanup(fail(MTO_EHIP, "hipEventCreate failed"));
  if (hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(fail(MTO_EHIP, "hipStreamCreate failed"));
  if (hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(MTO_EHIP, "hipEventCreate failed"));
  if (P->prm.precond != MTO_PRECOND_JACOBI && (rc = build_mg(P, I))) return cleanup(rc);
  if (P->prm.precond == MTO_PRECOND_MG_ASM && (rc = build_asm(P, I))) return cleanup(rc);
  if ((rc = rebuild_tiles(P))) return cleanup(rc);
  HIP_TRY(hipDeviceSynchronize());
  *out = P;
  return MTO_OK;
}

// ---- enqueue helpers (all launches on st; usable under stream capture) ----

// One group's product: its stored element matrices when it has them (they
// hold this design's moduli once the set-up or mto_autotune assembled them),
// else the contraction.
void enq_elem_group(mto_plan* P, const GroupHost& g, const double* xin, int mode, int it_k, hipStream_t st,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  if (g.stored && P->prm.kernel_path == MTO_PATH_MFMA)
    launch_elem_stored(P->gdev(g), P->d_tiles, xin, P->pcg(), mode, it_k, st, ev0, ev1);
  else
    launch_elem(P->gdev(g), P->prm.kernel_path, P->d_tiles, P->E, xin, P->pcg(), mode, it_k, st, ev0, ev1);
}

// Switches a group to stored element matrices (allocated on first use).
int ensure_stored(mto_plan* P, GroupHost& g) {
  if (!g.kst) {
    int rc = dev_alloc(P, &g.kst, (size_t)asm_ntp_of(g.p) * g.npad);
    if (rc) return rc;
  }
  g.stored = 1;
  return MTO_OK;
}

void enq_assemble_stored(mto_plan* P, hipStream_t st) {
  if (P->prm.kernel_path != MTO_PATH_MFMA) return;
  for (auto& g : P->groups)
    if (g.stored) launch_elem_assemble(P->gdev(g), P->E, g.kst, st);
}

void enq_elem_all(mto_plan* P, const double* xin, int mode, int it_k, hipStream_t st) {
  const PcgDev s = P->pcg();
  if (P->fused && P->prm.kernel_path == MTO_PATH_MFMA) {
    launch_elem_fused(P->d_groups_cur, P->d_tiles, P->fused_tile_begin, P->fused_n_tiles, P->n_sys > 1 ? 8 : 0,
                      P->fused_lds, P->E, xin, s, mode, it_k, st);
    return;
  }
  for (auto& g : P->groups) enq_elem_group(P, g, xin, mode, it_k, st);
}

void enq_residual(mto_plan* P, hipStream_t st);

// Per design, the level operators (level-1 operator, Galerkin products, l1
// diagonals) and the coarsest grid's factor.
void enq_mg_factor(mto_plan* P, hipStream_t st) {
  const MgHost& M = P->mg;
  launch_mg_assemble1(M.instc(1), M.inst_count[0], M.elems, M.kv, P->E, M.vfree, M.A, M.mask, st);
  launch_mg_l1(M.instc(1), M.inst_count[0], M.A, M.dinv, st);
  for (int l = 2; l <= M.L; ++l) {
    launch_mg_rap(M.instc(l), M.inst_count[l - 1], M.A, M.mask, st);
    launch_mg_l1(M.instc(l), M.inst_count[l - 1], M.A, M.dinv, st);
  }
  launch_mg_coarse_factor(M.coarse_instc(), P->n_inst, M.coarse_bmax, M.A, M.band, st);
}

// The coarsest grid's dense inverse from its factor.
void enq_mg_inverse(mto_plan* P, hipStream_t st) {
  const MgHost& M = P->mg;
  launch_mg_coarse_inverse(M.coarse_instc(), P->n_inst, M.coarse_nmax, M.band, M.scr, M.dense, st);
}

// z = M r: one V-cycle from z = D0^-1 r (already in z), l1-Jacobi pre- and
// post-smoothing on every level, dense solve on the coarsest; the last kernel
// also forms the partial sums of r.z.
void enq_elem_all(mto_plan* P, const double* xin, int mode, int it_k, hipStream_t st);

// The coarse-grid correction shared by both smoothers: restrict r - A0 z
// (A0 z in the slots) to the vertex grid, one V-cycle over levels 1..L,
// prolongate and add to z.
void enq_coarse_correction(mto_plan* P, hipStream_t st) {
  const MgHost& M = P->mg;
  const PcgDev s = P->pcg();
  launch_mg_restrict0(M.sysc(1), M.sys_count[0], s, M.vfree, M.dinv, M.r, M.e, st);
  for (int l = 2; l <= M.L; ++l)
    launch_mg_resid_restrict(M.isysc(l), M.isys_count[l - 1], s, M.A, M.mask, M.dinv, M.r, M.e, st);
  launch_mg_coarse_solve(M.coarse_isysc(), P->n_inst, M.coarse_nmax, s, M.dense, M.r, M.e2, st);
  // level 1 also injects its correction into z (with one level, prolong0 does)
  for (int l = M.L - 1; l >= 1; --l)
    launch_mg_prolong_smooth(M.isysc(l), M.isys_count[l - 1], s, M.A, M.mask, M.dinv, M.r, M.e, M.e2,
                             l == 1 ? M.vfree : nullptr, st);
  if (M.L == 1) launch_mg_prolong0(M.sysc(1), M.sys_count[0], s, M.vfree, M.e2, st);
}

// The slots hold K z from before the coarse-grid correction, which changed z
// at vertex DOFs only (by the values also left in q): add K[:, vertex] of
// that change, so the slots hold K z after it.
void enq_vertex_update(mto_plan* P, hipStream_t st) {
  const PcgDev s = P->pcg();
  if (P->prm.kernel_path == MTO_PATH_PLAIN) {  // the comparison path keeps its full product
    enq_elem_all(P, P->z, ELEM_APPLY_RUNNING, 0, st);
    return;
  }
  for (auto& g : P->groups) launch_elem_vertex(P->gdev(g), P->d_tiles, P->E, P->q, s, st);
}

// z = M r: one V-cycle.  Level-0 smoothing is Jacobi-type (z = D0^-1 r is
// already in z; l1 or damped post-sweep) or the element-block Schwarz
// smoother (pre: z = w B r; post: z += w B (r - A0 z)).  The last kernel also
// forms the partial sums of r.z.
void enq_vcycle(mto_plan* P, int it_k, int init, hipStream_t st) {
  const PcgDev s = P->pcg();
  if (P->prm.precond == MTO_PRECOND_MG_ASM) {
    for (auto& g : P->groups) launch_asm_apply(P->gdev(g), P->d_tiles, g.binv, P->r, 0, s, P->slots2, P->asm_omega, st);
    launch_asm_z(s, P->slots2, st);
    enq_elem_all(P, P->z, ELEM_APPLY_RUNNING, 0, st);
    enq_coarse_correction(P, st);
    enq_vertex_update(P, st);
    // post-smoothing: the residual r - A0 z is formed in the gather
    for (auto& g : P->groups) launch_asm_apply(P->gdev(g), P->d_tiles, g.binv, P->r, 1, s, P->slots2, P->asm_omega, st);
    launch_asm_post(s, P->slots2, it_k, init, st);
    return;
  }
  enq_elem_all(P, P->z, ELEM_APPLY_RUNNING, 0, st);
  enq_coarse_correction(P, st);
  enq_vertex_update(P, st);
  launch_mg_post0(s, it_k, init, st);
}

void enq_setup(mto_plan* P, const double* rho, const double* u0, hipStream_t st) {
  const PcgDev s = P->pcg();
  // the densities are checked here; k_sys_setup then stops every system if one is invalid
  launch_fill_i32(P->bad_rho, 0, 1, st);
  launch_fill_i32(P->dd_ok, 0, P->n_sys, st);  // new moduli: no residual in the slots is valid
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st, P->bad_rho);
  enq_assemble_stored(P, st);
  const bool mg = P->prm.precond != MTO_PRECOND_JACOBI;
  // l1-Jacobi level-0 smoother of MTO_PRECOND_MG unless a damping factor is set
  const bool l1 = P->prm.precond == MTO_PRECOND_MG && !(P->prm.mg_omega > 0.0);
  const bool damped = P->prm.precond == MTO_PRECOND_MG && !l1;
  for (auto& g : P->groups)
    launch_diag_elem(P->gdev(g), P->d_tiles, P->E, P->slots, P->d_sys, l1 ? g.kabs : g.kdiag, st);
  launch_dinv(s, P->dinv, damped ? P->prm.mg_omega : 1.0, st);
  // The multigrid set-up depends only on the moduli, as do the Schwarz block
  // inverses.  The coarsest factor is one workgroup on a serial chain that
  // runs several times slower when it shares its CU with the block inverses,
  // which fill every CU; so the level operators and the factor run first,
  // alone, and the dense inverse (many waves) then runs as a branch on the
  // side stream (under capture, a parallel branch of the graph) beside the
  // block inverses, joining before the first V-cycle.  Nothing on this
  // stream until the join touches the buffers of that branch.
  if (mg) {
    enq_mg_factor(P, st);
    (void)hipEventRecord(P->fork_ev, st);
    (void)hipStreamWaitEvent(P->side_stream, P->fork_ev, 0);
    enq_mg_inverse(P, P->side_stream);
    (void)hipEventRecord(P->join_ev, P->side_stream);
  }
  if (P->prm.precond == MTO_PRECOND_MG_ASM)
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
      const GroupHost& g = P->groups[gi];
      launch_asm_block(P->gdev(g), (int)gi, P->d_groups, g.nbr, P->d_el_group, P->d_el_col, P->E, g.binv, st);
    }
  // PCG iterates on the correction x (from 0); the solution is xs_hi + xs_lo
  launch_fill(P->x, 0.0, P->n_vec, st);
  launch_fill(P->xs_lo, 0.0, P->n_vec, st);
  if (u0) {
    launch_gather_free(s, P->f2f, u0, P->xs_hi, st);
    enq_residual(P, st);
    launch_init(s, 2, st);
  } else {
    launch_fill(P->xs_hi, 0.0, P->n_vec, st);
    launch_init(s, 0, st);
  }
  launch_sys_setup(s, P->prm.rtol, 0, st);
  if (mg) {
    (void)hipStreamWaitEvent(st, P->join_ev, 0);
    enq_vcycle(P, 0, 1, st);
  }
}

// G PCG iterations; the last one checks for residual replacement (systems
// whose recursive residual has come near its rounding floor) before its
// V-cycle, which then forms z from the replaced residual.
void enq_chunk(mto_plan* P, int G, hipStream_t st) {
  const PcgDev s = P->pcg();
  std::vector<GroupDev> gd;
  for (auto& g : P->groups) gd.push_back(P->gdev(g));
  for (int k = 0; k < G; ++k) {
    enq_elem_all(P, P->p, ELEM_PCG, k, st);
    launch_dof1(s, k, st);
    launch_dof2(s, k, st);
    if (k == G - 1)
      launch_replace(gd.data(), (int)gd.size(), P->d_tiles, P->E, s, P->xs_hi, P->xs_lo, P->slots_lo, k, st);
    if (P->prm.precond != MTO_PRECOND_JACOBI) enq_vcycle(P, k, 0, st);
  }
  launch_advance(s, G, st);
}

// True residual f - K x in double-double (then rounded): the FP64 product
// K x cannot resolve residuals below about eps || |K| |x| ||, which for the
// contrast E_min / E0 = 1e-9 lies above 1e-11 || f ||.
void enq_residual(mto_plan* P, hipStream_t st) {
  std::vector<GroupDev> gd;
  for (auto& g : P->groups) gd.push_back(P->gdev(g));
  launch_residual_dd(gd.data(), (int)gd.size(), P->d_tiles, P->E, P->pcg(), P->xs_hi, P->xs_lo, P->slots_lo, st);
}

// End of a PCG cycle: fold the correction into the refined solution, then
// the accurate residual of the result.
void enq_cycle_end(mto_plan* P, hipStream_t st) {
  launch_accumulate(P->pcg(), P->xs_hi, P->xs_lo, st);
  enq_residual(P, st);
}

// Iterative refinement: PCG continues from x with the accurate residual.
void enq_restart(mto_plan* P, hipStream_t st) {
  launch_init(P->pcg(), 2, st);
  launch_sys_setup(P->pcg(), P->prm.rtol, 1, st);
  if (P->prm.precond != MTO_PRECOND_JACOBI) enq_vcycle(P, 0, 1, st);
}

void enq_outputs(mto_plan* P, double* u, double* c, double* g, hipStream_t st) {
  const PcgDev s = P->pcg();
  launch_compliance(s, c, st);
  launch_fill(u, 0.0, P->n_u, st);
  launch_scatter_full(s, P->f2f, P->xs_hi, u, st);
  if (g)
    for (auto& gr : P->groups) launch_sens(P->gdev(gr), P->d_tiles, P->dE, P->xs_hi, P->xs_hi, g, P->d_sys, st);
}

int capture(mto_plan* P, hipGraphExec_t* exec, const std::function<void(hipStream_t)>& body) {
  if (*exec) {
    (void)hipGraphExecDestroy(*exec);
    *exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  body(P->cap_stream);
  hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
  if (e != hipSuccess) return fail(MTO_EHIP, std::string("stream capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MTO_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return MTO_OK;
}

// The chunk graphs: G iterations, and a short one of max(2, G / 4) for the
// last iterations before convergence (both even: the parity of it_base).
int ensure_chunk_graph(mto_plan* P) {
  const int G = P->prm.iters_per_launch;
  if (P->chunk_exec && P->small_exec && P->chunk_G == G) return MTO_OK;
  const int Gs = std::max(2, (G / 4) & ~1);
  int rc = capture(P, &P->chunk_exec, [&](hipStream_t st) { enq_chunk(P, G, st); });
  if (rc) return rc;
  if ((rc = capture(P, &P->small_exec, [&](hipStream_t st) { enq_chunk(P, Gs, st); }))) return rc;
  P->chunk_G = G;
  P->small_G = Gs;
  return MTO_OK;
}

// Runs PCG iterations until every system has stopped or the cap is reached.
// Each chunk ends by reporting the number of running systems and the largest
// rr / tol2 among them.  The host keeps at most two full chunks queued past
// the last report, as a plain pipeline would, but no more iterations than
// the log-linear extrapolation of that ratio to 1 asks for; near the end it
// queues short chunks, so that few iterations are launched after the last
// system has stopped (those return at once but still cost their launches).
// r0 is rr / tol2 at iteration 0 when the caller knows it (else <= 0).
int iterate(mto_plan* P, hipStream_t st, int64_t& launched, double r0) {
  int rc = ensure_chunk_graph(P);
  if (rc) return rc;
  const int G = P->chunk_G, Gs = P->small_G;
  int64_t cap = P->prm.max_iter;
  if (cap <= 0) {
    int64_t mx = 0;
    for (int i = 0; i < P->n_inst; ++i) mx = std::max(mx, P->n_free[i]);
    cap = std::max<int64_t>(20 * mx, 1000);
  }
  struct Pending {
    int slot;
    int64_t end;
  };
  Pending pend[N_PROG];
  int head = 0, n_pend = 0, next_slot = 0;
  int64_t queued = 0, known = 0;
  // reports (iteration, rr / tol2) of this cycle while systems still run
  std::vector<std::pair<int64_t, double>> hist;
  if (r0 > 1.0 && std::isfinite(r0)) hist.emplace_back(0, r0);
  auto launch = [&](bool full) -> int {
    const int slot = next_slot;
    next_slot = (next_slot + 1) % N_PROG;
    HIP_TRY(hipGraphLaunch(full ? P->chunk_exec : P->small_exec, st));
    HIP_TRY(hipMemcpyAsync(P->h_prog + 2 * slot, P->progress, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(P->ev[slot], st));
    queued += full ? G : Gs;
    pend[(head + n_pend) % N_PROG] = Pending{slot, queued};
    ++n_pend;
    return MTO_OK;
  };
  double rate = 0.0;
  while (true) {
    int64_t target = known + 2 * G;
    rate = 0.0;
    if (hist.size() >= 2) {
      // the latest report against the newest one at least G iterations older
      size_t j = hist.size() - 2;
      while (j > 0 && hist.back().first - hist[j].first < G) --j;
      rate = std::log(hist[j].second / hist.back().second) / double(hist.back().first - hist[j].first);
    }
    if (!(rate > 0.0 && std::isfinite(rate))) rate = P->rate_hint;
    if (rate > 0.0 && !hist.empty()) {
      const double need = std::ceil(std::log(hist.back().second) / rate);  // >= 1: the ratio is > 1
      if (need < double(cap)) target = std::min(target, hist.back().first + (int64_t)need);
    }
    if (queued < target && queued < cap && n_pend < N_PROG) {
      if ((rc = launch(target - queued >= G))) return rc;
      continue;
    }
    if (n_pend == 0) break;  // the cap is reached
    const Pending pd = pend[head];
    head = (head + 1) % N_PROG;
    --n_pend;
    HIP_TRY(hipEventSynchronize(P->ev[pd.slot]));
    known = pd.end;
    const double running = P->h_prog[2 * pd.slot], far = P->h_prog[2 * pd.slot + 1];
    if (running == 0.0) break;
    if (far > 1.0 && std::isfinite(far)) hist.emplace_back(pd.end, far);
  }
  if (rate > 0.0 && std::isfinite(rate)) P->rate_hint = rate;
  launched = queued;
  // no synchronisation here: the caller's next work (the true residual and
  // its copy to the host) follows these chunks in stream order
  return MTO_OK;
}

struct SysResult {
  std::vector<int32_t> status, iters;
  std::vector<double> out;
};

int fetch(mto_plan* P, hipStream_t st, SysResult& R) {
  R.status.resize(P->n_sys);
  R.iters.resize(P->n_sys);
  R.out.resize(4 * (size_t)P->n_sys);
  // one copy of the per-system block into pinned memory
  HIP_TRY(hipMemcpyAsync(P->h_sysblk, P->sysblk, 5 * (size_t)P->n_sys * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int32_t* hs = reinterpret_cast<const int32_t*>(P->h_sysblk);
  std::memcpy(R.status.data(), hs, P->n_sys * sizeof(int32_t));
  std::memcpy(R.iters.data(), hs + P->n_sys, P->n_sys * sizeof(int32_t));
  std::memcpy(R.out.data(), P->h_sysblk + P->n_sys, 4 * (size_t)P->n_sys * sizeof(double));
  return MTO_OK;
}

// The shared solve driver; `graphs` selects captured setup/residual/outputs.
int run_solve(mto_plan* P, const double* rho, double* u, double* c, double* g, const double* u0, hipStream_t st,
              mto_solve_stats* stats, bool graphs) {
  auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (graphs) {
    HIP_TRY(hipGraphLaunch(P->setup_exec, st));
  } else {
    enq_setup(P, rho, u0, st);
    if ((rc = check_launch("setup"))) return rc;
  }
  SysResult R;
  int restarts = 0;
  std::vector<int32_t> iters_total(P->n_sys, 0);
  std::vector<double> prev_res(P->n_sys, 0.0);
  int final_status = MTO_OK;
  // rr / tol2 at the start of a cycle: 1 / rtol^2 from x = 0, else from the
  // true residuals of the last cycle (unknown for a given initial guess)
  const double rtol2 = P->prm.rtol * P->prm.rtol;
  double r0 = u0 ? 0.0 : 1.0 / rtol2;
  while (true) {
    int64_t launched = 0;
    if ((rc = iterate(P, st, launched, r0))) return rc;
    if (graphs) {
      HIP_TRY(hipGraphLaunch(P->resid_exec, st));
    } else {
      enq_cycle_end(P, st);
      if ((rc = check_launch("residual"))) return rc;
    }
    if ((rc = fetch(P, st, R))) return rc;
    bool any_breakdown = false, any_running = false, need_restart = false, any_bad = false;
    for (int s = 0; s < P->n_sys; ++s) {
      iters_total[s] += R.iters[s];
      if (R.status[s] == SYS_BREAKDOWN) any_breakdown = true;
      else if (R.status[s] == SYS_RUNNING) any_running = true;
      else if (R.status[s] == SYS_BADINPUT) any_bad = true;
      const double ff = R.out[4 * s + 0], res = R.out[4 * s + 2];
      // Restart from the true residual while it misses rtol and the last
      // restart still halved it; once it stalls it sits at the FP64 rounding
      // floor of K u and further restarts cannot lower it.
      const bool misses = res > P->prm.rtol * P->prm.rtol * ff;
      const bool improving = restarts == 0 || res < 0.25 * prev_res[s];
      if (R.status[s] == SYS_CONVERGED && misses && improving) need_restart = true;
      prev_res[s] = res;
      if (s == 0) r0 = 0.0;
      if (ff > 0.0) r0 = std::max(r0, res / (rtol2 * ff));
    }
    if (any_bad) {
      final_status = MTO_EINVAL;
      break;
    }
    if (any_breakdown) {
      final_status = MTO_EBREAKDOWN;
      break;
    }
    if (any_running) {
      final_status = MTO_ENOCONV;
      break;
    }
    if (!need_restart || restarts >= P->prm.max_restarts) {
      // The stop test is the true residual: a system whose residual still
      // misses rtol (stalled at the rounding floor, or out of restarts) has
      // not converged, whatever its PCG recurrence reported.
      for (int s = 0; s < P->n_sys; ++s)
        if (!(R.out[4 * s + 2] <= rtol2 * R.out[4 * s + 0])) final_status = MTO_ENOCONV;  // NaN fails too
      break;
    }
    ++restarts;
    if (graphs) {
      HIP_TRY(hipGraphLaunch(P->restart_exec, st));
    } else {
      enq_restart(P, st);
      if ((rc = check_launch("restart"))) return rc;
    }
  }
  if (graphs) {
    HIP_TRY(hipGraphLaunch(P->out_exec, st));
  } else {
    enq_outputs(P, u, c, g, st);
    if ((rc = check_launch("outputs"))) return rc;
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (stats) {
    stats->status = final_status;
    stats->n_systems = P->n_sys;
    stats->restarts = restarts;
    stats->max_iterations = 0;
    for (int s = 0; s < P->n_sys; ++s) {
      stats->max_iterations = std::max(stats->max_iterations, iters_total[s]);
      if (stats->iterations) stats->iterations[s] = iters_total[s];
      if (stats->true_rel_residual) {
        const double ff = R.out[4 * s + 0], res = R.out[4 * s + 2];
        stats->true_rel_residual[s] = ff > 0 ? std::sqrt(res / ff) : std::sqrt(res);
      }
    }
    stats->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (final_status == MTO_EINVAL) return fail(MTO_EINVAL, "rho: a density is not finite or lies outside [0, 1]");
  if (final_status == MTO_EBREAKDOWN) return fail(MTO_EBREAKDOWN, "PCG breakdown (p^T K p <= 0 or non-finite)");
  if (final_status == MTO_ENOCONV)
    return fail(MTO_ENOCONV, "the true residual of a system misses rtol (PCG reached max_iter, or the "
                             "residual stalled above rtol after its restarts)");
  return MTO_OK;
}

}  // namespace

// ============================== C ABI ======================================

extern "C" {

const char* mto_last_error(void) { return g_err.c_str(); }

const char* mto_version(void) { return "mto-mi355x 0.1 (gfx950)"; }

int mto_plan_create(const mto_problem* prob, const mto_params* params, mto_plan** out) {
  g_err.clear();
  return build_plan(prob, 1, params, out);
}

int mto_batch_plan_create(const mto_problem* probs, int32_t n_instances, const mto_params* params,
                          mto_plan** out) {
  g_err.clear();
  return build_plan(probs, n_instances, params, out);
}

int mto_plan_info(const mto_plan* P, mto_plan_info_t* info) {
  if (!P || !info) return fail(MTO_EINVAL, "NULL argument");
  info->n_instances = P->n_inst;
  info->n_systems = P->n_sys;
  info->n_groups = (int32_t)P->groups.size();
  info->reserved = 0;
  info->n_cells = P->n_cells_tot;
  info->n_u = P->n_u;
  info->n_g = P->n_g;
  info->n_free_total = P->n_vec;
  info->n_elements = P->n_elements;
  double fl = 0.0;
  for (auto& g : P->groups) fl += g.flops;
  info->flops_per_matvec = fl;
  return MTO_OK;
}

int mto_instance_info(const mto_plan* P, int32_t i, int64_t* cell_off, int64_t* n_cells, int64_t* u_off,
                      int64_t* n_dof, int64_t* g_off, int64_t* c_off, int64_t* n_free, int32_t* n_load_cases) {
  if (!P || i < 0 || i >= P->n_inst) return fail(MTO_EINVAL, "bad plan or instance index");
  if (cell_off) *cell_off = P->cell_off[i];
  if (n_cells) *n_cells = P->n_cells[i];
  if (u_off) *u_off = P->u_off[i];
  if (n_dof) *n_dof = P->n_dof[i];
  if (g_off) *g_off = P->g_off[i];
  if (c_off) *c_off = P->c_off[i];
  if (n_free) *n_free = P->n_free[i];
  if (n_load_cases) *n_load_cases = P->L[i];
  return MTO_OK;
}

int mto_solve(mto_plan* P, const double* rho, double* u, double* c, double* g, const double* u0, void* stream,
              mto_solve_stats* stats) {
  g_err.clear();
  if (!P || !rho || !u || !c) return fail(MTO_EINVAL, "NULL plan, rho, u or c");
  return run_solve(P, rho, u, c, g, u0, (hipStream_t)stream, stats, false);
}

int mto_batch_capture(mto_plan* P, const double* rho, double* u, double* c, double* g, void* stream) {
  g_err.clear();
  if (!P || !rho || !u || !c) return fail(MTO_EINVAL, "NULL plan, rho, u or c");
  (void)stream;
  int rc;
  if ((rc = capture(P, &P->setup_exec, [&](hipStream_t st) { enq_setup(P, rho, nullptr, st); }))) return rc;
  if ((rc = capture(P, &P->resid_exec, [&](hipStream_t st) { enq_cycle_end(P, st); }))) return rc;
  if ((rc = capture(P, &P->restart_exec, [&](hipStream_t st) { enq_restart(P, st); }))) return rc;
  if ((rc = capture(P, &P->out_exec, [&](hipStream_t st) { enq_outputs(P, u, c, g, st); }))) return rc;
  if ((rc = ensure_chunk_graph(P))) return rc;
  P->bound = true;
  P->b_rho = rho;
  P->b_u = u;
  P->b_c = c;
  P->b_g = g;
  return MTO_OK;
}

int mto_batch_replay(mto_plan* P, void* stream, mto_solve_stats* stats) {
  g_err.clear();
  if (!P) return fail(MTO_EINVAL, "NULL plan");
  if (!P->bound || !P->setup_exec) return fail(MTO_EINVAL, "no captured buffers: call mto_batch_capture first");
  return run_solve(P, P->b_rho, P->b_u, P->b_c, P->b_g, nullptr, (hipStream_t)stream, stats, true);
}

int mto_apply_stiffness(mto_plan* P, const double* rho, const double* x, double* y, void* stream) {
  g_err.clear();
  if (!P || !rho || !x || !y) return fail(MTO_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const PcgDev s = P->pcg();
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  enq_assemble_stored(P, st);
  launch_gather_free(s, P->f2f, x, P->q, st);
  enq_elem_all(P, P->q, ELEM_APPLY, 0, st);
  launch_fill(y, 0.0, P->n_u, st);
  launch_assemble_to_full(s, P->f2f, y, 0, st);
  return check_launch("apply_stiffness");
}

}  // extern "C"

// ---- allocation-free stiffness product --------------------------------------
// Scratch of mto_apply_stiffness_noalloc: the cell moduli and their
// derivatives, the gathered x and the element slots, in one file-scope device
// array that every call on a device shares.  Host code uses the array only
// through the device address hipGetSymbolAddress gives for it on each device.
namespace {
constexpr int64_t NOALLOC_DOUBLES = MTO_NOALLOC_SCRATCH_BYTES / 8;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
std::mutex g_scratch_mu;
double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on device dev (the current device), looked
// up once per device.
int scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(MTO_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MTO_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return MTO_OK;
}
}  // namespace

extern "C" {

int mto_apply_stiffness_noalloc(mto_plan* P, const double* rho, const double* x, double* y, void* stream) {
  g_err.clear();
  if (!P || !rho || !x || !y) return fail(MTO_EINVAL, "NULL argument");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device) return fail(MTO_EINVAL, "the current device is not the plan's device");
  const int64_t need = 2 * P->n_cells_tot + P->n_vec + P->n_slots_tot;
  if (need > NOALLOC_DOUBLES)
    return fail(MTO_EINVAL, "mto_apply_stiffness_noalloc: the plan needs " + std::to_string(8 * need) +
                                " bytes of scratch, more than the " + std::to_string(MTO_NOALLOC_SCRATCH_BYTES) +
                                " the library holds");
  double* base = nullptr;
  int rc = scratch_address(dev, &base);
  if (rc) return rc;
  double* E = base;
  double* dE = E + P->n_cells_tot;
  double* q = dE + P->n_cells_tot;
  double* slots = q + P->n_vec;
  hipStream_t st = (hipStream_t)stream;
  PcgDev s = P->pcg();
  s.q = q;
  s.slots = slots;
  launch_simp(rho, E, dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  launch_gather_free(s, P->f2f, x, q, st);
  // slots that no element writes (missing neighbours) must read as zero; the
  // array keeps the previous call's contents
  launch_fill(slots, 0.0, P->n_slots_tot, st);
  for (auto& g : P->groups) launch_elem(P->gdev(g), P->prm.kernel_path, P->d_tiles, E, q, s, ELEM_APPLY, 0, st);
  launch_fill(y, 0.0, P->n_u, st);
  launch_assemble_to_full(s, P->f2f, y, 0, st);
  return check_launch("apply_stiffness_noalloc");
}

int mto_sensitivity(mto_plan* P, const double* rho, const double* u, double* g, void* stream) {
  g_err.clear();
  if (!P || !rho || !u || !g) return fail(MTO_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const PcgDev s = P->pcg();
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  launch_gather_free(s, P->f2f, u, P->q, st);
  for (auto& gr : P->groups) launch_sens(P->gdev(gr), P->d_tiles, P->dE, P->q, P->q, g, P->d_sys, st);
  return check_launch("sensitivity");
}

// Tables and index arrays of the QR-error indicator, once per plan.
static int qr_setup(mto_plan* P) {
  if (P->qr_ready) return MTO_OK;
  int rc;
  for (auto& g : P->groups) {
    const int q = g.p + 1, nq = ne_of(q), nt = nq * (nq + 1) / 2;
    const std::vector<double> ks = subcell_tables(q, g.d, P->prm.nu);
    std::vector<double> packed((size_t)g.S * nt);
    for (int s = 0; s < g.S; ++s)
      for (int i = 0; i < nq; ++i)
        for (int j = 0; j <= i; ++j) packed[(size_t)s * nt + i * (i + 1) / 2 + j] = ks[((size_t)s * nq + i) * nq + j];
    if ((rc = dev_upload(P, &g.qtab, packed)) || (rc = dev_upload(P, &g.d_eid, g.eid_h)) ||
        (rc = dev_upload(P, &g.d_einst, g.einst_h)))
      return rc;
  }
  const int n = P->n_inst;
  std::vector<int32_t> sys0(n), L(n), nel(n, 0);
  std::vector<int64_t> eoff(n);
  for (auto& g : P->groups)
    for (int i = 0; i < n; ++i) nel[i] += g.inst_begin[i + 1] - g.inst_begin[i];
  int64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    sys0[i] = (int32_t)P->c_off[i];  // systems are numbered instance-major, like c
    L[i] = P->L[i];
    eoff[i] = acc;
    acc += (int64_t)L[i] * nel[i];
  }
  if ((rc = dev_upload(P, &P->d_qr_sys0, sys0)) || (rc = dev_upload(P, &P->d_qr_L, L)) ||
      (rc = dev_upload(P, &P->d_qr_nel, nel)) || (rc = dev_upload(P, &P->d_qr_eoff, eoff)))
    return rc;
  P->qr_ready = true;
  return MTO_OK;
}

// Per-instance output offsets (as for the QR indicator) and the element
// lookup of the refinement indicators, once per plan.
static int adapt_setup(mto_plan* P) {
  if (P->ad_ready) return MTO_OK;
  const int n = P->n_inst;
  std::vector<int64_t> base(n + 1, 0);
  for (int i = 0; i < n; ++i) base[i + 1] = base[i] + (int64_t)P->inst_nelx[i] * P->inst_nely[i];
  std::vector<int32_t> elg(base[n], -1), elc(base[n], -1);
  std::vector<GroupDev> gd;
  for (size_t g = 0; g < P->groups.size(); ++g) {
    const GroupHost& G = P->groups[g];
    for (size_t k = 0; k < G.eid_h.size(); ++k) {
      elg[base[G.einst_h[k]] + G.eid_h[k]] = (int32_t)g;
      elc[base[G.einst_h[k]] + G.eid_h[k]] = (int32_t)k;
    }
    gd.push_back(P->gdev(G));
  }
  base.pop_back();
  int rc;
  if ((rc = dev_upload(P, &P->d_ad_groups, gd)) || (rc = dev_upload(P, &P->d_ad_elgroup, elg)) ||
      (rc = dev_upload(P, &P->d_ad_elcol, elc)) || (rc = dev_upload(P, &P->d_ad_nelx, P->inst_nelx)) ||
      (rc = dev_upload(P, &P->d_ad_nely, P->inst_nely)) || (rc = dev_upload(P, &P->d_ad_base, base)))
    return rc;
  P->ad_ready = true;
  return MTO_OK;
}

static AdaptDev adapt_dev(const mto_plan* P) {
  AdaptDev a{};
  a.groups = P->d_ad_groups;
  a.el_group = P->d_ad_elgroup;
  a.el_col = P->d_ad_elcol;
  a.nelx = P->d_ad_nelx;
  a.nely = P->d_ad_nely;
  a.el_base = P->d_ad_base;
  a.inst_eoff = P->d_qr_eoff;
  return a;
}

int mto_kelly_indicator(mto_plan* P, const double* u, double* gamma, void* stream) {
  g_err.clear();
  if (!P || !u || !gamma) return fail(MTO_EINVAL, "NULL argument");
  int rc;
  if ((rc = qr_setup(P)) || (rc = adapt_setup(P))) return rc;
  hipStream_t st = (hipStream_t)stream;
  launch_gather_free(P->pcg(), P->f2f, u, P->q, st);
  int nel_max = 0;
  for (int i = 0; i < P->n_inst; ++i) nel_max = std::max(nel_max, P->inst_nelx[i] * P->inst_nely[i]);
  launch_kelly(adapt_dev(P), P->d_sys, P->n_sys, nel_max, P->q, gamma, st);
  return check_launch("kelly_indicator");
}

int mto_density_indicator(mto_plan* P, const double* rho, int32_t cycle, double alpha, double beta, double rho_min,
                          double rho_max, double* gamma, void* stream) {
  g_err.clear();
  if (!P || !rho || !gamma) return fail(MTO_EINVAL, "NULL argument");
  if (cycle < 1 || !(rho_max > rho_min) || !std::isfinite(alpha) || !std::isfinite(beta))
    return fail(MTO_EINVAL, "density indicator: cycle >= 1 and rho_max > rho_min required");
  int rc;
  if ((rc = qr_setup(P)) || (rc = adapt_setup(P))) return rc;
  DensityBounds b{};
  b.avg = 0.5 * (rho_max + rho_min);
  const double s = b.avg * std::exp(-beta * (cycle - 1));
  b.rl = rho_min + (1.0 - alpha) * s;
  b.ru = rho_max - (1.0 - alpha) * s;
  b.cl = rho_min + alpha * s;
  b.cu = rho_max - alpha * s;
  launch_density_indicator(adapt_dev(P), rho, b, gamma, P->n_elements, (hipStream_t)stream);
  return check_launch("density_indicator");
}

int mto_qr_error(mto_plan* P, const double* rho, const double* u, double* eps, void* stream) {
  g_err.clear();
  if (!P || !rho || !u || !eps) return fail(MTO_EINVAL, "NULL argument");
  int rc = qr_setup(P);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const PcgDev s = P->pcg();
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  launch_gather_free(s, P->f2f, u, P->q, st);
  for (auto& g : P->groups) {
    QrGroupDev qd{};
    qd.p = g.p;
    qd.d = g.d;
    qd.S = g.S;
    qd.npad = g.npad;
    qd.n_elems = g.n_elems;
    qd.tab = g.qtab;
    qd.gidx = g.gidx;
    qd.cell = g.cell;
    qd.eid = g.d_eid;
    qd.einst = g.d_einst;
    const std::vector<double> t = qr_load_transfer(g.p);
    for (int k = 0; k <= MTO_MAX_P; ++k) qd.t[k] = k < (int)t.size() ? t[k] : 0.0;
    launch_qr(qd, P->E, P->q, P->d_sys, P->d_qr_sys0, P->d_qr_L, P->d_qr_eoff, P->d_qr_nel, eps, st);
  }
  return check_launch("qr_error");
}

int mto_jacobi_diagonal(mto_plan* P, const double* rho, double* diag, void* stream) {
  g_err.clear();
  if (!P || !rho || !diag) return fail(MTO_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const PcgDev s = P->pcg();
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  for (auto& g : P->groups) launch_diag_elem(P->gdev(g), P->d_tiles, P->E, P->slots, P->d_sys, g.kdiag, st);
  int64_t acc = 0;
  for (int i = 0; i < P->n_inst; ++i) acc += P->n_dof[i];
  launch_fill(diag, 0.0, acc, st);
  launch_assemble_to_full(s, P->f2f, diag, 1, st);
  return check_launch("jacobi_diagonal");
}

int mto_adjoint_sensitivity(mto_plan* P, const double* rho, const double* u, const double* lam, double* g,
                            void* stream) {
  g_err.clear();
  if (!P || !rho || !u || !lam || !g) return fail(MTO_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const PcgDev s = P->pcg();
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  launch_gather_free(s, P->f2f, u, P->q, st);
  launch_gather_free(s, P->f2f, lam, P->z, st);
  for (auto& gr : P->groups) launch_sens(P->gdev(gr), P->d_tiles, P->dE, P->q, P->z, g, P->d_sys, st);
  return check_launch("adjoint_sensitivity");
}

int mto_weighted_sensitivity(mto_plan* P, const double* g, const double* w, double* out, void* stream) {
  g_err.clear();
  if (!P || !g || !w || !out) return fail(MTO_EINVAL, "NULL argument");
  launch_weighted_sens(g, w, out, P->d_inst_cell_off, P->d_inst_g_off, P->d_inst_c_off, P->d_inst_L, P->n_inst,
                       P->n_cells_tot, (hipStream_t)stream);
  return check_launch("weighted_sensitivity");
}

int mto_set_tile(mto_plan* P, int32_t p, int32_t d, int32_t ncol, int32_t ks) {
  g_err.clear();
  if (P && ks == -1) {  // the fused product: one launch over every group
    P->fused = true;
    return rebuild_tiles(P);
  }
  if (P && ks == -2) {  // stored element matrices for the group(s)
    P->fused = false;
    bool any = false;
    for (auto& g : P->groups)
      if (p <= 0 || (g.p == p && g.d == d)) {
        int rc = ensure_stored(P, g);
        if (rc) return rc;
        any = true;
      }
    if (!any) return fail(MTO_EINVAL, "no group with this (p, d)");
    return rebuild_tiles(P);
  }
  if (!P || (ncol != 1 && ncol != 2 && ncol != 4) || ks < 0 || ks > 8)
    return fail(MTO_EINVAL, "ncol must be 1, 2 or 4 and ks -2..8");
  P->fused = false;
  if (ks == 0 && ncol == 4) return fail(MTO_EINVAL, "the LDS-staged contraction takes ncol 1 or 2");
  for (auto& g : P->groups)
    if (p <= 0 || (g.p == p && g.d == d)) {
      if (ks == 0) {
        if (g.p < 3) {
          if (p > 0) return fail(MTO_EINVAL, "the LDS-staged contraction needs p >= 3");
          continue;  // all groups: the others keep their shape
        }
        if (elem_lds_staged_bytes(g.p, ncol) > ELEM_LDS_STAGED_LIMIT)
          return fail(MTO_EINVAL, "tile shape exceeds the LDS limit");
        g.lds_nc = ncol;
        g.stored = 0;
        continue;
      }
      const int k = std::min<int>(ks, g.S);
      if (elem_lds_bytes(g.p, ncol, k) > ELEM_LDS_LIMIT) return fail(MTO_EINVAL, "tile shape exceeds the LDS limit");
      g.ncol = ncol;
      g.waves = k;
      g.lds_nc = 0;
      g.stored = 0;
    }
  return rebuild_tiles(P);
}

int mto_autotune(mto_plan* P, const double* rho, const char* cache_path, void* stream, char* report,
                 int32_t report_len) {
  g_err.clear();
  if (!P || !rho) return fail(MTO_EINVAL, "NULL argument");
  if (P->prm.kernel_path != MTO_PATH_MFMA) return MTO_OK;
  hipStream_t st = (hipStream_t)stream;
  std::string arch = "unknown";
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) {
      arch = prop.gcnArchName;
      const size_t colon = arch.find(':');
      if (colon != std::string::npos) arch.resize(colon);
    }
  }
  std::map<TileKey, TileChoice> cache;
  if (cache_path && !read_tile_cache(cache_path, cache))
    return fail(MTO_EINVAL, std::string("autotune cache: cannot parse ") + cache_path);
  launch_simp(rho, P->E, P->dE, P->n_cells_tot, P->prm.E0, P->prm.Emin, P->prm.q, st);
  launch_fill(P->q, 1.0, P->n_vec, st);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::string rep;
  bool changed = false;
  const int cand_nc[3] = {1, 2, 4};
  const int cand_ks[5] = {0, 1, 2, 4, 8};  // 0: the LDS-staged contraction
  for (auto& g : P->groups) {
    const TileKey key{arch, g.p, g.d, size_class(g.flops / (2.0 * g.S * g.ne * g.ne))};
    auto hit = cache.find(key);
    if (hit != cache.end() && hit->second.ks == -2 && P->prm.stored_matrices) {
      int rc = ensure_stored(P, g);
      if (rc) return rc;
      char line[200];
      snprintf(line, sizeof line,
               "p=%d d=%d ncol=1 ks=-2: cached (stored element matrices; %s, %d columns class, %.3f us when tuned)\n",
               g.p, g.d, arch.c_str(), key.size_class, hit->second.us);
      rep += line;
      continue;
    }
    g.stored = 0;
    if (hit != cache.end() && hit->second.ks == -2) hit = cache.end();  // stored matrices not allowed: time shapes
    if (hit != cache.end() && hit->second.ks == 0 && g.p >= 3 &&
        elem_lds_staged_bytes(g.p, hit->second.ncol) <= ELEM_LDS_STAGED_LIMIT) {
      g.lds_nc = hit->second.ncol;
      char line[200];
      snprintf(line, sizeof line, "p=%d d=%d ncol=%d ks=0: cached (%s, %d columns class, %.3f us when tuned)\n", g.p,
               g.d, g.lds_nc, arch.c_str(), key.size_class, hit->second.us);
      rep += line;
      continue;
    }
    if (hit != cache.end() && hit->second.ks > 0 &&
        elem_lds_bytes(g.p, hit->second.ncol, std::min(hit->second.ks, g.S)) <= ELEM_LDS_LIMIT) {
      g.lds_nc = 0;
      g.ncol = hit->second.ncol;
      g.waves = std::min(hit->second.ks, g.S);
      char line[200];
      snprintf(line, sizeof line, "p=%d d=%d ncol=%d ks=%d: cached (%s, %d columns class, %.3f us when tuned)\n", g.p,
               g.d, g.ncol, g.waves, arch.c_str(), key.size_class, hit->second.us);
      rep += line;
      continue;
    }
    double best = 1e30;
    int best_nc = g.ncol, best_ks = g.waves;
    for (int nc : cand_nc)
      for (int ks : cand_ks) {
        if (ks > 0 && (ks > g.S || elem_lds_bytes(g.p, nc, ks) > ELEM_LDS_LIMIT)) continue;
        if (ks > 0 && ((nc == 4 && g.p >= 2) || (nc == 2 && g.p == 4))) continue;  // register spills
        if (ks == 0 && (g.p < 3 || nc == 4 || elem_lds_staged_bytes(g.p, nc) > ELEM_LDS_STAGED_LIMIT)) continue;
        g.lds_nc = ks == 0 ? nc : 0;
        g.ncol = ks == 0 ? 1 : nc;
        g.waves = ks == 0 ? 1 : ks;
        int rc = rebuild_tiles(P);
        if (rc) return rc;
        const GroupDev gd = P->gdev(g);
        const PcgDev s = P->pcg();
        for (int w = 0; w < 3; ++w) launch_elem(gd, P->prm.kernel_path, P->d_tiles, P->E, P->q, s, ELEM_APPLY, 0, st);
        const int reps = 20;
        HIP_TRY(hipEventRecord(e0, st));
        for (int w = 0; w < reps; ++w) launch_elem(gd, P->prm.kernel_path, P->d_tiles, P->E, P->q, s, ELEM_APPLY, 0, st);
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        const double t = ms / reps;
        char line[160];
        snprintf(line, sizeof line, "p=%d d=%d ncol=%d ks=%d: %.3f us (%.1f GF/s)\n", g.p, g.d, nc, ks, 1e3 * t,
                 g.flops / (t * 1e6));
        rep += line;
        if (t < best) {
          best = t;
          best_nc = nc;
          best_ks = ks;
        }
      }
    if (g.p >= 3 && P->prm.stored_matrices) {  // stored element matrices: assembled for these moduli, then timed
      int rc = ensure_stored(P, g);
      if (rc) return rc;
      rc = rebuild_tiles(P);
      if (rc) return rc;
      launch_elem_assemble(P->gdev(g), P->E, g.kst, st);
      for (int w = 0; w < 3; ++w) enq_elem_group(P, g, P->q, ELEM_APPLY, 0, st);
      const int reps = 20;
      HIP_TRY(hipEventRecord(e0, st));
      for (int w = 0; w < reps; ++w) enq_elem_group(P, g, P->q, ELEM_APPLY, 0, st);
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      const double tt = ms / reps;
      char line[160];
      snprintf(line, sizeof line, "p=%d d=%d ncol=1 ks=-2: %.3f us (stored element matrices)\n", g.p, g.d, 1e3 * tt);
      rep += line;
      g.stored = 0;
      if (tt < best) {
        best = tt;
        best_nc = 1;
        best_ks = -2;
      }
    }
    g.stored = best_ks == -2 ? 1 : 0;
    g.lds_nc = best_ks == 0 ? best_nc : 0;
    g.ncol = best_ks <= 0 ? 1 : best_nc;
    g.waves = best_ks <= 0 ? 1 : best_ks;
    cache[key] = TileChoice{best_nc, best_ks, 1e3 * best};
    changed = true;
  }
  // one launch for all groups (the fused product) or one per group (the
  // stored element matrices, when chosen, for these moduli)
  enq_assemble_stored(P, st);
  {
    int64_t cols = 0;
    for (auto& g : P->groups) cols += (int64_t)(g.flops / (2.0 * g.S * g.ne * g.ne));
    const TileKey key{arch, 0, (int)P->groups.size(), size_class((double)cols)};
    auto hit = cache.find(key);
    if (hit != cache.end()) {
      P->fused = hit->second.ncol == 1;
    } else {
      double tm[2] = {0.0, 0.0};
      for (int f = 0; f < 2; ++f) {
        P->fused = f == 1;
        int rc = rebuild_tiles(P);
        if (rc) return rc;
        for (int w = 0; w < 3; ++w) enq_elem_all(P, P->q, ELEM_APPLY, 0, st);
        const int reps = 20;
        HIP_TRY(hipEventRecord(e0, st));
        for (int w = 0; w < reps; ++w) enq_elem_all(P, P->q, ELEM_APPLY, 0, st);
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        tm[f] = ms / reps;
      }
      P->fused = tm[1] < tm[0];
      char line[160];
      snprintf(line, sizeof line, "all groups: one launch per group %.3f us, one fused launch %.3f us\n", 1e3 * tm[0],
               1e3 * tm[1]);
      rep += line;
      cache[key] = TileChoice{P->fused ? 1 : 2, 0, 1e3 * std::min(tm[0], tm[1])};
      changed = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    char line[96];
    snprintf(line, sizeof line, "product: %s\n", P->fused ? "fused (one launch for all groups)" : "one launch per group");
    rep += line;
  }
  for (auto& g : P->groups) {
    char line[96];
    if (g.stored)
      snprintf(line, sizeof line, "p=%d d=%d ncol=1 ks=-2: chosen\n", g.p, g.d);
    else
      snprintf(line, sizeof line, "p=%d d=%d ncol=%d ks=%d: chosen\n", g.p, g.d, g.lds_nc ? g.lds_nc : g.ncol,
               g.lds_nc ? 0 : g.waves);
    rep += line;
  }
  int rc = rebuild_tiles(P);
  if (rc) return rc;
  if (cache_path && changed && !write_tile_cache(cache_path, cache))
    return fail(MTO_EHIP, std::string("autotune cache: cannot write ") + cache_path);
  if (report && report_len > 0) {
    snprintf(report, (size_t)report_len, "%s", rep.c_str());
  }
  return check_launch("autotune");
}

int mto_time_contraction(mto_plan* P, const double* rho, int32_t reps, int32_t in_loop, void* stream,
                         double* ms_per_matvec) {
  g_err.clear();
  if (!P || !rho || !ms_per_matvec || reps < 1 || (in_loop != 0 && in_loop != 1))
    return fail(MTO_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  enq_setup(P, rho, nullptr, st);
  int rc = check_launch("time_contraction setup");
  if (rc) return rc;
  if (!in_loop) {
    // PCG state of iteration 0 (x = 0, p = 0, beta = 0): each launch is the
    // search-direction product of the first iteration, identical every time.
    for (int w = 0; w < 3; ++w) enq_elem_all(P, P->p, ELEM_PCG, 0, st);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    for (int w = 0; w < reps; ++w) enq_elem_all(P, P->p, ELEM_PCG, 0, st);
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_matvec = (double)ms / reps;
    return check_launch("time_contraction");
  }
  // Inside the iteration: `reps` PCG iterations run eagerly from x = 0, the
  // same kernels in the same order as a captured chunk, so the products see
  // the caches the vector kernels leave behind.  Each product kernel carries
  // its own start/end events on its dispatch packet.
  const PcgDev s = P->pcg();
  const int G = P->prm.iters_per_launch;
  const size_t ng = P->groups.size();
  std::vector<hipEvent_t> ev(2 * ng * (size_t)reps, nullptr);
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  const bool fused = P->fused && P->prm.kernel_path == MTO_PATH_MFMA;
  for (int i = 0; i < reps; ++i) {
    const int k = i % G;
    if (fused) {
      hipEvent_t* e = &ev[2 * (ng * i)];
      launch_elem_fused(P->d_groups_cur, P->d_tiles, P->fused_tile_begin, P->fused_n_tiles, P->n_sys > 1 ? 8 : 0,
                        P->fused_lds, P->E, P->p, s, ELEM_PCG, k, st, e[0], e[1]);
    } else {
      for (size_t gi = 0; gi < ng; ++gi) {
        auto& g = P->groups[gi];
        hipEvent_t* e = &ev[2 * (ng * i + gi)];
        enq_elem_group(P, g, P->p, ELEM_PCG, k, st, e[0], e[1]);
      }
    }
    launch_dof1(s, k, st);
    launch_dof2(s, k, st);
    if (P->prm.precond != MTO_PRECOND_JACOBI) enq_vcycle(P, k, 0, st);
    if (k == G - 1 || i == reps - 1) launch_advance(s, k + 1, st);
  }
  HIP_TRY(hipStreamSynchronize(st));
  double total = 0.0;
  for (size_t j = 0; j < ng * (size_t)reps; ++j) {
    const GroupHost& gj = P->groups[j % ng];
    if (fused ? (j % ng != 0 || P->fused_n_tiles == 0) : (gj.stored ? gj.ms_n_tiles : gj.n_tiles) == 0)
      continue;  // nothing launched, events never recorded
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
    total += ms;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  *ms_per_matvec = total / reps;
  return check_launch("time_contraction");
}

void mto_plan_destroy(mto_plan* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  destroy_graphs(P);
  for (auto& a : P->allocs)
    if (a.ptr) (void)hipFree(a.ptr);
  if (P->h_prog) (void)hipHostFree(P->h_prog);
  if (P->h_sysblk) (void)hipHostFree(P->h_sysblk);
  for (int k = 0; k < N_PROG; ++k)
    if (P->ev[k]) (void)hipEventDestroy(P->ev[k]);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
  if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
  if (P->join_ev) (void)hipEventDestroy(P->join_ev);
  delete P;
}

}  // extern "C"
