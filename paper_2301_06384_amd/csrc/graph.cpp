// graph_kernel_init: validation of the CSR Laplacian (Sec. 2.1, eq. of the
// generalised Laplacian), conversion to difference form, optional BFS
// relabelling for gather locality, and upload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <vector>

#include "gk_internal.h"

namespace gk {

static void check_device() {
  int dev = 0;
  GK_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  GK_HIP(hipGetDeviceProperties(&prop, dev));
  const std::string arch(prop.gcnArchName);
  if (arch.find("gfx950") == std::string::npos)
    throw Error{GK_EDEVICE, "library built for gfx950, device is " + arch};
}

// Host-side validated, preprocessed copy (caller node order).
struct HostLap {
  int64_t n = 0;
  std::vector<int64_t> rp;     // off-diagonal CSR
  std::vector<int32_t> ci;
  std::vector<double> w;       // w_ij = -L_ij > 0
  std::vector<double> c;       // diagonal excess
  double lambda_max = 0;
  bool unit = false;
};

static HostLap validate(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                        uint32_t flags) {
  GK_REQUIRE(n >= 1, GK_EINVAL, "n must be >= 1");
  GK_REQUIRE(n < (int64_t(1) << 31), GK_EINVAL, "n must be < 2^31");
  GK_REQUIRE(row_ptr && col_idx, GK_EINVAL, "row_ptr and col_idx must not be NULL");
  const bool unit = (flags & GK_UNIT_WEIGHTS) != 0;
  GK_REQUIRE(unit || vals, GK_EINVAL, "vals is NULL without GK_UNIT_WEIGHTS");
  GK_REQUIRE(row_ptr[0] == 0, GK_EINVAL, "row_ptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    GK_REQUIRE(row_ptr[i + 1] >= row_ptr[i], GK_EINVAL, "row_ptr not nondecreasing");
  const int64_t nnz = row_ptr[n];
  double maxabs = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const int32_t j = col_idx[p];
      GK_REQUIRE(j >= 0 && j < n, GK_EINVAL, "column index out of range in row " + std::to_string(i));
      if (p > row_ptr[i]) GK_REQUIRE(col_idx[p - 1] < j, GK_EINVAL, "columns not strictly increasing in row " + std::to_string(i));
      if (!unit) {
        GK_REQUIRE(std::isfinite(vals[p]), GK_EINVAL, "non-finite value");
        maxabs = std::max(maxabs, std::fabs(vals[p]));
      }
    }
  }
  (void)nnz;
  HostLap H;
  H.n = n;
  H.unit = unit;
  H.rp.assign(n + 1, 0);
  H.c.assign(n, 0.0);
  const double symtol = 1e-14 * maxabs;
  // off-diagonal part, symmetry and sign checks
  for (int64_t i = 0; i < n; ++i) {
    double diag = 0.0, sumw = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const int32_t j = col_idx[p];
      const double v = unit ? -1.0 : vals[p];
      if (j == i) {
        diag = unit ? 0.0 : v;
        continue;
      }
      // structural + numerical symmetry: find (j, i)
      const int32_t* b = col_idx + row_ptr[j];
      const int32_t* e = col_idx + row_ptr[j + 1];
      const int32_t* f = std::lower_bound(b, e, (int32_t)i);
      if (f == e || *f != i) {
        if (v == 0.0) continue;   // explicit zero without partner: no edge
        throw Error{GK_ENOTSYM, "missing symmetric entry (" + std::to_string(j) + "," + std::to_string(i) + ")"};
      }
      if (!unit) {
        const double vt = vals[row_ptr[j] + (f - b)];
        if (std::fabs(v - vt) > symtol)
          throw Error{GK_ENOTSYM, "L(" + std::to_string(i) + "," + std::to_string(j) + ") != L(" +
                                      std::to_string(j) + "," + std::to_string(i) + ")"};
      }
      if (v > 0.0) throw Error{GK_ENOTLAP, "positive off-diagonal entry in row " + std::to_string(i)};
      if (v == 0.0) continue;   // explicit zero: not an edge
      H.ci.push_back(j);
      H.w.push_back(-v);
      sumw += -v;
    }
    H.rp[i + 1] = (int64_t)H.ci.size();
    if (unit) {
      H.c[i] = 0.0;
    } else {
      double ex = diag - sumw;
      if (std::fabs(ex) <= 1e-14 * (std::fabs(diag) + sumw)) ex = 0.0;
      if (ex < 0.0 && !(flags & GK_ASSUME_PSD))
        throw Error{GK_ENOTLAP, "negative diagonal excess in row " + std::to_string(i) +
                                    " (not diagonally dominant; pass GK_ASSUME_PSD)"};
      H.c[i] = ex;
    }
    H.lambda_max = std::max(H.lambda_max, std::fabs(sumw + H.c[i]) + sumw);
  }
  GK_REQUIRE((int64_t)H.ci.size() < (int64_t(1) << 31) - 1, GK_EINVAL, "too many nonzeros for int32 offsets");
  if (H.lambda_max <= 0.0) H.lambda_max = 1.0;   // edgeless graph with zero diagonal
  return H;
}

// BFS (Cuthill-McKee) order: new node k is old node order[k].  Components are
// visited in order of their lowest-degree unvisited node.
static std::vector<int64_t> bfs_order(const HostLap& H) {
  const int64_t n = H.n;
  std::vector<int64_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int64_t> byDeg(n);
  for (int64_t i = 0; i < n; ++i) byDeg[i] = i;
  std::stable_sort(byDeg.begin(), byDeg.end(),
                   [&](int64_t a, int64_t b) { return (H.rp[a + 1] - H.rp[a]) < (H.rp[b + 1] - H.rp[b]); });
  std::vector<int64_t> nb;
  for (int64_t s0 : byDeg) {
    if (seen[s0]) continue;
    size_t head = order.size();
    order.push_back(s0);
    seen[s0] = 1;
    while (head < order.size()) {
      const int64_t u = order[head++];
      nb.clear();
      for (int64_t p = H.rp[u]; p < H.rp[u + 1]; ++p)
        if (!seen[H.ci[p]]) {
          seen[H.ci[p]] = 1;
          nb.push_back(H.ci[p]);
        }
      std::stable_sort(nb.begin(), nb.end(),
                       [&](int64_t a, int64_t b) { return (H.rp[a + 1] - H.rp[a]) < (H.rp[b + 1] - H.rp[b]); });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  return order;
}

static void upload(gk_graph* g, const HostLap& H, const std::vector<int64_t>* order) {
  const int64_t n = H.n;
  std::vector<int32_t> rp(n + 1, 0), ci;
  std::vector<double> w64, d64(n), d32(n);
  std::vector<float> w32;
  std::vector<int64_t> iperm;
  if (order) {
    iperm.assign(n, 0);
    for (int64_t k = 0; k < n; ++k) iperm[(*order)[k]] = k;
  }
  ci.reserve(H.ci.size());
  if (!H.unit) {
    w64.reserve(H.w.size());
    w32.reserve(H.w.size());
  }
  std::vector<std::pair<int32_t, double>> row;
  int maxrow = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = order ? (*order)[k] : k;
    row.clear();
    for (int64_t p = H.rp[i]; p < H.rp[i + 1]; ++p)
      row.push_back({(int32_t)(order ? iperm[H.ci[p]] : H.ci[p]), H.unit ? 1.0 : H.w[p]});
    std::sort(row.begin(), row.end());
    double s64 = 0.0, s32 = 0.0;
    for (auto& e : row) {
      ci.push_back(e.first);
      if (!H.unit) {
        w64.push_back(e.second);
        const float f = (float)e.second;
        w32.push_back(f);
        s32 += (double)f;
      }
      s64 += e.second;
    }
    if (H.unit) s32 = s64;
    d64[k] = s64 + H.c[i];
    d32[k] = s32 + H.c[i];
    rp[k + 1] = (int32_t)ci.size();
    maxrow = std::max(maxrow, (int)row.size());
  }
  // per-XCD row ranges of equal cost for the products
  {
    const double tot = (double)ci.size() + 3.0 * (double)n;
    int64_t i = 0;
    double acc = 0.0;
    g->xr[0] = 0;
    for (int x = 1; x < 8; ++x) {
      const double goal = tot * x / 8.0;
      while (i < n && acc + 0.5 * (rp[i + 1] - rp[i] + 3.0) <= goal) {
        acc += rp[i + 1] - rp[i] + 3.0;
        ++i;
      }
      g->xr[x] = i;
    }
    g->xr[8] = n;
  }
  std::vector<int32_t> hub;
  for (int64_t k = 0; k < n; ++k)
    if (rp[k + 1] - rp[k] > g->hub_min) hub.push_back((int32_t)k);
  g->nhub = (int64_t)hub.size();
  g->n = n;
  g->nnz = (int64_t)ci.size();
  g->unit = H.unit;
  g->lambda_max = H.lambda_max;
  g->max_row = maxrow;
  auto put = [](auto*& dst, const auto& src) {
    using T = typename std::decay<decltype(src[0])>::type;
    size_t bytes = std::max<size_t>(src.size() * sizeof(T), 256);
    void* p = nullptr;
    GK_HIP(hipMalloc(&p, bytes));
    if (!src.empty()) GK_HIP(hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    dst = static_cast<T*>(p);
  };
  put(g->rp, rp);
  put(g->ci, ci);
  if (!H.unit) {
    put(g->w64, w64);
    put(g->w32, w32);
  }
  put(g->d64, d64);
  put(g->d32, d32);
  put(g->hub, hub);
  if (order) {
    g->reordered = true;
    put(g->d_perm, *order);
    put(g->d_iperm, iperm);
    g->h_iperm = iperm;
  }
}

}  // namespace gk

extern "C" {

int graph_kernel_init(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                      uint32_t flags, gk_graph** out) {
  if (!out) return GK_EINVAL;
  *out = nullptr;
  gk_graph* g = nullptr;
  try {
    gk::HostLap H = gk::validate(n, row_ptr, col_idx, vals, flags);
    gk::check_device();
    g = new gk_graph();
    GK_HIP(hipGetDevice(&g->device));
    if (flags & GK_REORDER) {
      std::vector<int64_t> order = gk::bfs_order(H);
      gk::upload(g, H, &order);
    } else {
      gk::upload(g, H, nullptr);
    }
    *out = g;
    return GK_OK;
  } catch (const gk::Error& e) {
    gk::set_detail(e.msg);
    if (g) graph_kernel_release(g);
    return e.code;
  } catch (const std::exception& e) {
    gk::set_detail(e.what());
    if (g) graph_kernel_release(g);
    return GK_ENOMEM;
  }
}

void graph_kernel_release(gk_graph* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)g->rp, (void*)g->ci, (void*)g->w64, (void*)g->w32, (void*)g->d64, (void*)g->d32,
                  (void*)g->d_perm, (void*)g->d_iperm, (void*)g->hub})
    if (p) (void)hipFree(p);
  delete g;
}

int gk_graph_info(const gk_graph* g, int64_t* n, int64_t* nnz_offdiag, double* lambda_max) {
  if (!g) return GK_EINVAL;
  if (n) *n = g->n;
  if (nnz_offdiag) *nnz_offdiag = g->nnz;
  if (lambda_max) *lambda_max = g->lambda_max;
  return GK_OK;
}

}  // extern "C"
