// Host-side numbering of one design instance: the conforming mixed-p space
// (minimum rule on edges), supports, free-DOF compaction, the slot layout of
// the deterministic scatter, and the load vectors.
//
// Global scalar functions, in this order (vector DOF = 2 id + component):
//   vertices              id = vy*(nelx+1) + vx
//   horizontal edges      edge h = vy*nelx + ex, modes 2..hdeg[h]
//   vertical edges        edge v = ey*(nelx+1) + vx, modes 2..vdeg[v]
//   element interiors     element e, modes (i, j), i, j in 2..p_e, i fastest
// An edge carries the modes 2..min(p) of its (one or two) elements, so the
// space is the conforming piecewise-Q_{p_e} space; the edge modes of the
// higher-order neighbour above that degree are absent.
//
// Scatter slots: every free DOF owns a fixed number of consecutive slots, one
// per element that can touch it: 4 for a vertex DOF (position 2 j_loc + i_loc,
// the corner of the element at that vertex), 2 for an edge DOF (position =
// the side of the edge the element lies on), 1 for an interior DOF.  Element
// kernels write each local result to its own slot with a plain store; the
// vector kernels sum a DOF's slots in a fixed order.  Free DOFs keep the full
// ordering, so free vertex DOFs come first, then edge DOFs, then interiors,
// and the first slot of free DOF i follows from i and the two counts.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <set>

#include "mto_internal.hpp"

namespace mto {

namespace {

int64_t slot_base(int64_t i, int64_t nfv, int64_t nfe) {
  if (i < nfv) return 4 * i;
  if (i < nfv + nfe) return 4 * nfv + 2 * (i - nfv);
  return 4 * nfv + 2 * nfe + (i - nfv - nfe);
}

}  // namespace

int build_instance(const mto_problem& prob, InstanceHost& I, std::string& err) {
  char buf[256];
  const int nelx = prob.mesh.nelx, nely = prob.mesh.nely;
  if (nelx < 1 || nely < 1 || (int64_t)nelx * nely > (1 << 26)) {
    err = "mesh size out of range";
    return MTO_EINVAL;
  }
  if (!prob.mesh.p || !prob.mesh.d) {
    err = "mesh p or d is NULL";
    return MTO_EINVAL;
  }
  if (prob.n_load_cases < 1 || prob.n_loads < 0 || (prob.n_loads > 0 && !prob.loads) ||
      prob.n_supports < 0 || (prob.n_supports > 0 && !prob.supports) || prob.n_springs < 0 ||
      (prob.n_springs > 0 && !prob.springs)) {
    err = "bad load or support arrays";
    return MTO_EINVAL;
  }
  const int nel = nelx * nely;
  I.nelx = nelx;
  I.nely = nely;
  I.L = prob.n_load_cases;
  I.p.assign(prob.mesh.p, prob.mesh.p + nel);
  I.d.assign(prob.mesh.d, prob.mesh.d + nel);
  I.cell_off.assign(nel + 1, 0);
  for (int e = 0; e < nel; ++e) {
    if (I.p[e] < 1 || I.p[e] > MTO_MAX_P || I.d[e] < 1 || I.d[e] > MTO_MAX_D) {
      snprintf(buf, sizeof buf, "element %d: p=%d d=%d out of range (p 1..%d, d 1..%d)", e, I.p[e], I.d[e],
               MTO_MAX_P, MTO_MAX_D);
      err = buf;
      return MTO_EINVAL;
    }
    I.cell_off[e + 1] = I.cell_off[e] + (int64_t)I.d[e] * I.d[e];
  }
  I.n_cells = I.cell_off[nel];
  auto P = [&](int ex, int ey) { return (int)I.p[(size_t)ey * nelx + ex]; };

  // edge degrees and scalar id offsets
  const int64_t nv = (int64_t)(nelx + 1) * (nely + 1);
  const int64_t nh = (int64_t)nelx * (nely + 1), nvv = (int64_t)(nelx + 1) * nely;
  std::vector<int> hdeg(nh), vdeg(nvv);
  std::vector<int64_t> hoff(nh), voff(nvv), ioff(nel);
  int64_t id = nv;
  for (int vy = 0; vy <= nely; ++vy)
    for (int ex = 0; ex < nelx; ++ex) {
      int dg = 1 << 30;
      if (vy > 0) dg = std::min(dg, P(ex, vy - 1));
      if (vy < nely) dg = std::min(dg, P(ex, vy));
      const int64_t h = (int64_t)vy * nelx + ex;
      hdeg[h] = dg;
      hoff[h] = id;
      id += dg - 1;
    }
  for (int ey = 0; ey < nely; ++ey)
    for (int vx = 0; vx <= nelx; ++vx) {
      int dg = 1 << 30;
      if (vx > 0) dg = std::min(dg, P(vx - 1, ey));
      if (vx < nelx) dg = std::min(dg, P(vx, ey));
      const int64_t v = (int64_t)ey * (nelx + 1) + vx;
      vdeg[v] = dg;
      voff[v] = id;
      id += dg - 1;
    }
  const int64_t first_edge_id = nv, first_interior_id = id;
  for (int e = 0; e < nel; ++e) {
    ioff[e] = id;
    id += (int64_t)(I.p[e] - 1) * (I.p[e] - 1);
  }
  I.n_scalar = id;
  I.n_dof = 2 * id;
  if (I.n_dof >= (int64_t)1 << 31) {
    err = "instance too large for 32-bit DOF indices";
    return MTO_EINVAL;
  }

  // supports
  std::vector<uint8_t> fixed(I.n_dof, 0);
  bool have_x = false, have_y = false;
  std::set<int> x_rows_y, y_rows_x;  // rigid-mode check: y of x-fixed vertices, x of y-fixed
  auto fix_vertex = [&](int vx, int vy, int mask) {
    const int64_t vid = (int64_t)vy * (nelx + 1) + vx;
    if (mask & 1) {
      fixed[2 * vid] = 1;
      have_x = true;
      x_rows_y.insert(vy);
    }
    if (mask & 2) {
      fixed[2 * vid + 1] = 1;
      have_y = true;
      y_rows_x.insert(vx);
    }
  };
  auto fix_ids = [&](int64_t first, int64_t count, int mask) {
    for (int64_t k = first; k < first + count; ++k) {
      if (mask & 1) fixed[2 * k] = 1;
      if (mask & 2) fixed[2 * k + 1] = 1;
    }
  };
  for (int s = 0; s < prob.n_supports; ++s) {
    const mto_support& S = prob.supports[s];
    if (S.comp_mask < 1 || S.comp_mask > 3) {
      snprintf(buf, sizeof buf, "support %d: comp_mask %d not in 1..3", s, S.comp_mask);
      err = buf;
      return MTO_EINVAL;
    }
    switch (S.kind) {
      case MTO_SUP_VERTEX:
        if (S.a < 0 || S.a > nelx || S.b < 0 || S.b > nely) {
          snprintf(buf, sizeof buf, "support %d: vertex (%d,%d) outside the mesh", s, S.a, S.b);
          err = buf;
          return MTO_EINVAL;
        }
        fix_vertex(S.a, S.b, S.comp_mask);
        break;
      case MTO_SUP_EDGE_LEFT:
      case MTO_SUP_EDGE_RIGHT: {
        const int vx = S.kind == MTO_SUP_EDGE_LEFT ? 0 : nelx;
        for (int vy = 0; vy <= nely; ++vy) fix_vertex(vx, vy, S.comp_mask);
        for (int ey = 0; ey < nely; ++ey) {
          const int64_t v = (int64_t)ey * (nelx + 1) + vx;
          fix_ids(voff[v], vdeg[v] - 1, S.comp_mask);
        }
        break;
      }
      case MTO_SUP_EDGE_BOTTOM:
      case MTO_SUP_EDGE_TOP: {
        const int vy = S.kind == MTO_SUP_EDGE_BOTTOM ? 0 : nely;
        for (int vx = 0; vx <= nelx; ++vx) fix_vertex(vx, vy, S.comp_mask);
        for (int ex = 0; ex < nelx; ++ex) {
          const int64_t h = (int64_t)vy * nelx + ex;
          fix_ids(hoff[h], hdeg[h] - 1, S.comp_mask);
        }
        break;
      }
      default:
        snprintf(buf, sizeof buf, "support %d: unknown kind %d", s, S.kind);
        err = buf;
        return MTO_EINVAL;
    }
  }
  // A rigid motion (a - theta y, b + theta x) is interpolated by the vertex
  // functions alone, so only vertex constraints can stop it; they do iff the
  // rows (1, 0, -y) / (0, 1, x) have rank 3.
  if (!(have_x && have_y && (x_rows_y.size() >= 2 || y_rows_x.size() >= 2))) {
    err = "supports leave a rigid-body mode free";
    return MTO_ESINGULAR;
  }

  // free numbering
  I.full_to_free.assign(I.n_dof, -1);
  I.free_to_full.clear();
  int64_t nf = 0, nfv = 0, nfe = 0, nfi = 0;
  for (int64_t k = 0; k < I.n_dof; ++k) {
    if (fixed[k]) continue;
    I.full_to_free[k] = (int32_t)nf++;
    I.free_to_full.push_back((int32_t)k);
    const int64_t sid = k / 2;
    if (sid < first_edge_id) ++nfv;
    else if (sid < first_interior_id) ++nfe;
    else ++nfi;
  }
  if (nf == 0) {
    err = "no free DOFs (every DOF is supported)";
    return MTO_EINVAL;
  }
  I.n_free = (int32_t)nf;
  I.nfv = (int32_t)nfv;
  I.nfe = (int32_t)nfe;
  I.nfi = (int32_t)nfi;
  I.n_slots = 4 * nfv + 2 * nfe + nfi;

  // element descriptors
  I.elem_dof_off.assign(nel + 1, 0);
  for (int e = 0; e < nel; ++e) I.elem_dof_off[e + 1] = I.elem_dof_off[e] + ne_of(I.p[e]);
  I.elem_free.assign(I.elem_dof_off[nel], -1);
  I.elem_slot.assign(I.elem_dof_off[nel], -1);
  for (int ey = 0; ey < nely; ++ey)
    for (int ex = 0; ex < nelx; ++ex) {
      const int e = ey * nelx + ex, pe = I.p[e], n1 = pe + 1;
      int32_t* fr = &I.elem_free[I.elem_dof_off[e]];
      int32_t* sl = &I.elem_slot[I.elem_dof_off[e]];
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          int64_t sid = -1;
          int pos = 0;
          if (i <= 1 && j <= 1) {
            sid = (int64_t)(ey + j) * (nelx + 1) + (ex + i);
            pos = 2 * j + i;
          } else if (j <= 1) {
            const int64_t h = (int64_t)(ey + j) * nelx + ex;
            if (i <= hdeg[h]) sid = hoff[h] + (i - 2);
            pos = j;
          } else if (i <= 1) {
            const int64_t v = (int64_t)ey * (nelx + 1) + ex + i;
            if (j <= vdeg[v]) sid = voff[v] + (j - 2);
            pos = i;
          } else {
            sid = ioff[e] + (int64_t)(j - 2) * (pe - 1) + (i - 2);
            pos = 0;
          }
          const int a = j * n1 + i;
          for (int c = 0; c < 2; ++c) {
            if (sid < 0) continue;
            const int32_t f = I.full_to_free[2 * sid + c];
            if (f < 0) continue;
            fr[2 * a + c] = f;
            sl[2 * a + c] = (int32_t)(slot_base(f, nfv, nfe) + pos);
          }
        }
    }

  // ground springs
  I.springs.clear();
  for (int k = 0; k < prob.n_springs; ++k) {
    const mto_spring& Sp = prob.springs[k];
    if (Sp.vx < 0 || Sp.vx > nelx || Sp.vy < 0 || Sp.vy > nely || Sp.comp < 0 || Sp.comp > 1 ||
        !(Sp.k > 0.0) || !std::isfinite(Sp.k)) {
      snprintf(buf, sizeof buf, "spring %d: vertex (%d,%d) comp %d k %g out of range", k, Sp.vx, Sp.vy, Sp.comp, Sp.k);
      err = buf;
      return MTO_EINVAL;
    }
    const int32_t f = I.full_to_free[2 * ((int64_t)Sp.vy * (nelx + 1) + Sp.vx) + Sp.comp];
    if (f < 0) {
      snprintf(buf, sizeof buf, "spring %d acts on a supported DOF", k);
      err = buf;
      return MTO_EINVAL;
    }
    I.springs.emplace_back(f, Sp.k);
  }

  // loads
  I.f.assign((size_t)I.L * nf, 0.0);
  for (int k = 0; k < prob.n_loads; ++k) {
    const mto_point_load& Ld = prob.loads[k];
    if (Ld.vx < 0 || Ld.vx > nelx || Ld.vy < 0 || Ld.vy > nely || Ld.load_case < 0 ||
        Ld.load_case >= I.L) {
      snprintf(buf, sizeof buf, "load %d: vertex (%d,%d) case %d out of range", k, Ld.vx, Ld.vy, Ld.load_case);
      err = buf;
      return MTO_EINVAL;
    }
    const int64_t vid = (int64_t)Ld.vy * (nelx + 1) + Ld.vx;
    const double fc[2] = {Ld.fx, Ld.fy};
    for (int c = 0; c < 2; ++c) {
      if (fc[c] == 0.0) continue;
      const int32_t f = I.full_to_free[2 * vid + c];
      if (f < 0) {
        snprintf(buf, sizeof buf, "load %d acts on a supported DOF", k);
        err = buf;
        return MTO_EINVAL;
      }
      I.f[(size_t)Ld.load_case * nf + f] += fc[c];
    }
  }
  return MTO_OK;
}

}  // namespace mto
