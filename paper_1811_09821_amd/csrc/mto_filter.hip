// Density filter of Sec. 2.2 (Eqs. (4)-(5)) on the density cells and its
// transpose for the chain rule.
//
// H is symmetric (H_ij = R - |c_i - c_j| is the same float either way round),
// so one pattern serves both directions: with s_i = 1 / sum_j H_ij,
//   apply:  y_i = s_i sum_j H_ij x_j            (W = diag(s) H)
//   grad:   y_i = sum_j H_ij (s_j x_j)          (W^T = H diag(s))
// The pattern is stored sliced by 64 rows (one wavefront): slice t holds its
// rows' k-th entries side by side at sp[t] + 64 k + lane, padded to the
// slice's longest row with zero weights pointing at the row itself, so each
// load of a wave is one contiguous run (256 B of indices, 512 B of weights)
// and no lane diverges.  Both directions are plain gathers: no atomics, bit-reproducible.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "mto_internal.hpp"

using namespace mto;

namespace {
constexpr int FSLICE = 64;  // rows per slice = wavefront width
}

struct mto_filter {
  int device = 0;
  double R = 0.0;
  int64_t n = 0, nnz = 0, stored = 0;
  int64_t* sp = nullptr;   // [n_slices + 1] slice starts (entries)
  int32_t* col = nullptr;  // [stored]
  double* h = nullptr;     // [stored] H_ij
  double* s = nullptr;     // [n] 1 / sum_j H_ij
};

namespace {

template <bool GRAD>
__global__ __launch_bounds__(256) void k_filter(const int64_t* __restrict__ sp, const int32_t* __restrict__ col,
                                                const double* __restrict__ h, const double* __restrict__ s,
                                                const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = i / FSLICE;
  const int lane = (int)(i % FSLICE);
  // slices past the end of the last one have no entries: sp is read only for t < n_slices
  if (i >= n) return;
  const int64_t b = sp[t], e = sp[t + 1];
  double acc = 0.0;
  for (int64_t k = b + lane; k < e; k += FSLICE) {
    const int32_t j = col[k];
    const double xj = GRAD ? s[j] * x[j] : x[j];
    acc = fma(h[k], xj, acc);
  }
  y[i] = GRAD ? acc : s[i] * acc;
}

template <class T>
int upload(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  if (hipMalloc((void**)dst, bytes) != hipSuccess) return set_error(MTO_ENOMEM, "hipMalloc failed (density filter)");
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return set_error(MTO_EHIP, "hipMemcpy failed (density filter)");
  return MTO_OK;
}

int launch(const mto_filter* F, bool grad, const double* x, double* y, void* stream) {
  if (F->n == 0) return MTO_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != F->device)
    return set_error(MTO_EINVAL, "density filter used on a device other than the one it was created on");
  const unsigned blocks = (unsigned)((F->n + 255) / 256);
  if (grad)
    hipLaunchKernelGGL(k_filter<true>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, F->sp, F->col, F->h, F->s, x,
                       y, F->n);
  else
    hipLaunchKernelGGL(k_filter<false>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, F->sp, F->col, F->h, F->s,
                       x, y, F->n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MTO_EHIP, std::string("density filter launch: ") + hipGetErrorString(e));
  return MTO_OK;
}

}  // namespace

static int filter_create(const mto_problem* probs, int32_t n_inst, double R, mto_filter** out) {
  if (!out) return set_error(MTO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || n_inst < 1) return set_error(MTO_EINVAL, "no problems");
  if (!(R > 0.0) || !std::isfinite(R)) return set_error(MTO_EINVAL, "filter radius must be positive and finite");
  // rows of H with global column indices, instance by instance (element-major, s = sy*d + sx)
  std::vector<int64_t> rowp{0};
  std::vector<int32_t> rcol;
  std::vector<double> rh, inv;
  int64_t base = 0;
  for (int i = 0; i < n_inst; ++i) {
    const mto_mesh& m = probs[i].mesh;
    if (m.nelx < 1 || m.nely < 1 || !m.d) return set_error(MTO_EINVAL, "instance " + std::to_string(i) + ": bad mesh");
    const int nel = m.nelx * m.nely;
    std::vector<int64_t> eoff(nel + 1, 0);
    for (int e = 0; e < nel; ++e) {
      if (m.d[e] < 1 || m.d[e] > MTO_MAX_D) return set_error(MTO_EINVAL, "instance " + std::to_string(i) + ": bad d");
      eoff[e + 1] = eoff[e] + (int64_t)m.d[e] * m.d[e];
    }
    if (base + eoff[nel] >= ((int64_t)1 << 31)) return set_error(MTO_EINVAL, "too many cells for 32-bit indices");
    auto centre = [&](int e, int s, double& x, double& y) {
      const int de = m.d[e], ex = e % m.nelx, ey = e / m.nelx, sx = s % de, sy = s / de;
      x = ex + (sx + 0.5) / de;
      y = ey + (sy + 0.5) / de;
    };
    // centres lie strictly inside their elements, so two cells k elements
    // apart (in x or y) are more than k - 1 apart: k <= ceil(R) suffices
    const int rr = (int)std::min<double>(std::ceil(R), (double)std::max(m.nelx, m.nely));
    std::vector<std::pair<int64_t, double>> nb;
    for (int e = 0; e < nel; ++e) {
      const int ex = e % m.nelx, ey = e / m.nelx;
      for (int s = 0; s < m.d[e] * m.d[e]; ++s) {
        double xi, yi;
        centre(e, s, xi, yi);
        nb.clear();
        for (int ey2 = std::max(0, ey - rr); ey2 <= std::min(m.nely - 1, ey + rr); ++ey2)
          for (int ex2 = std::max(0, ex - rr); ex2 <= std::min(m.nelx - 1, ex + rr); ++ex2) {
            const int e2 = ey2 * m.nelx + ex2;
            for (int s2 = 0; s2 < m.d[e2] * m.d[e2]; ++s2) {
              double xj, yj;
              centre(e2, s2, xj, yj);
              const double dx = xi - xj, dy = yi - yj;
              const double dist = (e2 == e && s2 == s) ? 0.0 : std::sqrt(dx * dx + dy * dy);
              if (dist < R) nb.emplace_back(base + eoff[e2] + s2, R - dist);
            }
          }
        std::sort(nb.begin(), nb.end());
        double sum = 0.0;
        for (auto& t : nb) sum += t.second;
        inv.push_back(1.0 / sum);
        for (auto& t : nb) {
          rcol.push_back((int32_t)t.first);
          rh.push_back(t.second);
        }
        rowp.push_back((int64_t)rcol.size());
      }
    }
    base += eoff[nel];
  }
  const int64_t n = base, nnz = (int64_t)rcol.size();
  // slice by 64 rows, entries of a slice interleaved by lane
  const int64_t nsl = (n + FSLICE - 1) / FSLICE;
  std::vector<int64_t> sp(nsl + 1, 0);
  for (int64_t t = 0; t < nsl; ++t) {
    int64_t wmax = 0;
    for (int64_t r = t * FSLICE; r < std::min(n, (t + 1) * FSLICE); ++r) wmax = std::max(wmax, rowp[r + 1] - rowp[r]);
    sp[t + 1] = sp[t] + wmax * FSLICE;
  }
  const int64_t stored = sp[nsl];
  std::vector<int32_t> col(stored);
  std::vector<double> h(stored, 0.0);
  for (int64_t t = 0; t < nsl; ++t) {
    const int64_t wd = (sp[t + 1] - sp[t]) / FSLICE;
    for (int lane = 0; lane < FSLICE; ++lane) {
      const int64_t r = t * FSLICE + lane;
      for (int64_t k = 0; k < wd; ++k) {
        const int64_t dst = sp[t] + k * FSLICE + lane;
        const bool real = r < n && k < rowp[r + 1] - rowp[r];
        // padding: zero weight on the row's own cell (or cell 0 past the end)
        col[dst] = real ? rcol[rowp[r] + k] : (int32_t)(r < n ? r : 0);
        h[dst] = real ? rh[rowp[r] + k] : 0.0;
      }
    }
  }
  mto_filter* F = new mto_filter();
  if (hipGetDevice(&F->device) != hipSuccess) {
    delete F;
    return set_error(MTO_EHIP, "hipGetDevice failed");
  }
  F->R = R;
  F->n = n;
  F->nnz = nnz;
  F->stored = stored;
  int rc;
  if ((rc = upload(&F->sp, sp)) || (rc = upload(&F->col, col)) || (rc = upload(&F->h, h)) ||
      (rc = upload(&F->s, inv))) {
    mto_filter_destroy(F);
    return rc;
  }
  *out = F;
  return MTO_OK;
}

extern "C" {

int mto_filter_create(const mto_problem* probs, int32_t n_inst, double R, mto_filter** out) {
  clear_error();
  try {
    return filter_create(probs, n_inst, R, out);
  } catch (const std::bad_alloc&) {
    return set_error(MTO_ENOMEM, "host memory exhausted building the density filter (radius too large?)");
  }
}

int mto_filter_apply(const mto_filter* F, const double* rho, double* rho_tilde, void* stream) {
  clear_error();
  if (!F || !rho || !rho_tilde) return set_error(MTO_EINVAL, "NULL argument");
  if (rho == rho_tilde) return set_error(MTO_EINVAL, "the filter cannot run in place");
  return launch(F, false, rho, rho_tilde, stream);
}

int mto_filter_grad(const mto_filter* F, const double* g_tilde, double* g, void* stream) {
  clear_error();
  if (!F || !g_tilde || !g) return set_error(MTO_EINVAL, "NULL argument");
  if (g == g_tilde) return set_error(MTO_EINVAL, "the filter cannot run in place");
  return launch(F, true, g_tilde, g, stream);
}

int mto_filter_info(const mto_filter* F, int64_t* n_cells, int64_t* nnz) {
  clear_error();
  if (!F) return set_error(MTO_EINVAL, "NULL filter");
  if (n_cells) *n_cells = F->n;
  if (nnz) *nnz = F->nnz;
  return MTO_OK;
}

void mto_filter_destroy(mto_filter* F) {
  if (!F) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(F->device);
  (void)hipDeviceSynchronize();
  void* bufs[] = {F->sp, F->col, F->h, F->s};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete F;
}

}  // extern "C"
