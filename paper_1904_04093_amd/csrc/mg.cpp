// Geometric multigrid V-cycle around GaBP contexts (Sec. 4 of the paper).
//
// Two-grid cycle applied recursively: pre-smoothing, residual, full-weighting restriction,
// coarse error equation solved by the next level (directly on the coarsest one), bilinear
// interpolation of the correction, post-smoothing. The smoother is GaBP used as an error
// correction scheme (Algorithm 3, run by each level's own context with its mode, schedule,
// precision and warm policy) or red-black Gauss-Seidel, the classical comparison smoother.
// Grids are vertex-centred with side n_l interior points and n_l = 2 n_{l+1} + 1; the
// coarse operators are rediscretisations supplied by the caller as contexts.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gabp_internal.h"
#include "graph.h"

using namespace gabp;

// A recorded V-cycle (+ residual norms to the host) and the message-buffer parities of the
// level contexts before and after it: replaying it must leave the contexts exactly as the
// eager cycle would.
struct MgGraph {
  const double* b = nullptr;
  const double* x = nullptr;
  bool reuse = false;   // the finest pre-smoothing takes the previous check's residual
  std::vector<int> before, after;
  hipGraphExec_t exec = nullptr;
};

struct mg_ctx {
  int levels = 0;
  std::vector<gabp_ctx*> lv;
  std::vector<int32_t> side;
  int smoother = 0, nu1 = 0, nu2 = 0;
  std::vector<double*> b, x, r;   // per level: rhs and iterate (levels >= 1), residual
  double* inv = nullptr;          // dense inverse of the coarsest operator, row-major
  int nc = 0;
  int cycles_run = 0;
  bool use_graphs = true;
  hipStream_t capture_stream = nullptr;
  std::vector<MgGraph> graphs;
};

namespace {

int invert_dense(std::vector<double>& a, int n, std::vector<double>& inv) {
  // Gauss-Jordan with partial pivoting on [A | I]
  inv.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(a[static_cast<size_t>(i) * n + c]) > std::fabs(a[static_cast<size_t>(piv) * n + c])) piv = i;
    if (a[static_cast<size_t>(piv) * n + c] == 0.0) return fail(GABP_ENUMERIC, "singular coarsest operator");
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[static_cast<size_t>(piv) * n + k], a[static_cast<size_t>(c) * n + k]);
        std::swap(inv[static_cast<size_t>(piv) * n + k], inv[static_cast<size_t>(c) * n + k]);
      }
    const double d = a[static_cast<size_t>(c) * n + c];
    for (int k = 0; k < n; ++k) {
      a[static_cast<size_t>(c) * n + k] /= d;
      inv[static_cast<size_t>(c) * n + k] /= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == c) continue;
      const double f = a[static_cast<size_t>(i) * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[static_cast<size_t>(i) * n + k] -= f * a[static_cast<size_t>(c) * n + k];
        inv[static_cast<size_t>(i) * n + k] -= f * inv[static_cast<size_t>(c) * n + k];
      }
    }
  }
  return GABP_OK;
}

int dense_of(gabp_ctx* c, std::vector<double>& A, hipStream_t s) {
  const Layout& L = c->L;
  const int n = L.n;
  std::vector<int32_t> sptr(L.nslices + 1), col(L.epad);
  std::vector<double> val(L.epad), diag(n);
  GABP_HIP(hipMemcpyAsync(sptr.data(), L.sptr, sptr.size() * 4, hipMemcpyDeviceToHost, s));
  GABP_HIP(hipMemcpyAsync(col.data(), L.col, col.size() * 4, hipMemcpyDeviceToHost, s));
  GABP_HIP(hipMemcpyAsync(val.data(), L.val, val.size() * 8, hipMemcpyDeviceToHost, s));
  GABP_HIP(hipMemcpyAsync(diag.data(), L.diag, diag.size() * 8, hipMemcpyDeviceToHost, s));
  GABP_HIP(hipStreamSynchronize(s));
  A.assign(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    A[static_cast<size_t>(j) * n + j] = diag[j];
    const int t = L.lane_of_row.empty() ? j : L.lane_of_row[j];
    const int sl = t / kSlice;
    const int w = (sptr[sl + 1] - sptr[sl]) / kSlice;
    for (int k = 0; k < w; ++k) {
      const int p = sptr[sl] + k * kSlice + t % kSlice;
      if (val[p] != 0.0) A[static_cast<size_t>(j) * n + col[p]] += val[p];
    }
  }
  return GABP_OK;
}

int smooth(mg_ctx* m, int l, const double* b, double* x, int nu, hipStream_t s,
           bool r_ready = false, bool x_zero = false) {
  if (nu <= 0) return GABP_OK;
  gabp_ctx* c = m->lv[l];
  if (m->smoother == 0) return smooth_from(c, b, x, nu, r_ready, x_zero, s);
  for (int it = 0; it < nu; ++it)
    for (int col = 0; col < 2; ++col) GABP_HIP(launch_rbgs(&c->L, m->side[l], col, b, x, s));
  return GABP_OK;
}

// x_zero: the coarse levels' error equations start from x = 0; x is then not read (and
// not cleared) unless the pre-smoother needs it (RB-GS, or no pre-smoothing)
int vcycle(mg_ctx* m, int l, const double* b, double* x, hipStream_t s, bool r_ready = false,
           bool x_zero = false) {
  int st;
  if (l == m->levels - 1) {
    GABP_HIP(launch_dense_matvec(m->nc, m->inv, b, x, s));
    return GABP_OK;
  }
  gabp_ctx* c = m->lv[l];
  const bool gabp_from_zero = x_zero && m->smoother == 0 && m->nu1 > 0;
  if (x_zero && !gabp_from_zero) GABP_HIP(launch_fill64(x, c->L.n, 0.0, s));
  if ((st = smooth(m, l, b, x, m->nu1, s, r_ready, gabp_from_zero)) != GABP_OK) return st;
  GABP_HIP(launch_residual(&c->L, c->L.val, b, x, nullptr, nullptr, m->r[l], c->partials,
                           c->nred, c->red, s, false));
  GABP_HIP(launch_restrict_fw(m->side[l + 1], m->r[l], m->b[l + 1], s));
  if ((st = vcycle(m, l + 1, m->b[l + 1], m->x[l + 1], s, false, true)) != GABP_OK) return st;
  GABP_HIP(launch_prolong_add(m->side[l + 1], m->x[l + 1], x, s));
  return smooth(m, l, b, x, m->nu2, s);
}

// host-side message state of every level (ping-pong parities, reset flags)
std::vector<int> parities(const mg_ctx* m) {
  std::vector<int> p;
  for (const gabp_ctx* c : m->lv) {
    p.push_back(c->parity);
    p.push_back(c->parity32);
    p.push_back(c->fresh64);
    p.push_back(c->fresh32);
  }
  return p;
}

void set_parities(mg_ctx* m, const std::vector<int>& p) {
  for (size_t l = 0; l < m->lv.size(); ++l) {
    m->lv[l]->parity = p[4 * l];
    m->lv[l]->parity32 = p[4 * l + 1];
    m->lv[l]->fresh64 = p[4 * l + 2] != 0;
    m->lv[l]->fresh32 = p[4 * l + 3] != 0;
  }
}

// One V-cycle followed by the finest residual's norms copied to the host (no wait). The
// check's residual b - A x is kept in the finest smoother's residual buffer: a solve's next
// cycle (reuse) starts its pre-smoothing from it instead of forming it again.
int enqueue_cycle(mg_ctx* m, const double* b, double* x, bool reuse, hipStream_t s) {
  int st = vcycle(m, 0, b, x, s, reuse && m->smoother == 0);
  if (st != GABP_OK) return st;
  gabp_ctx* c = m->lv[0];
  GABP_HIP(launch_residual(&c->L, c->L.val, b, x, nullptr, nullptr, c->r, c->partials,
                           c->nred, c->red, s));
  GABP_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  return GABP_OK;
}

// Run one cycle; from the second cycle on (every Lt phase done, every buffer allocated) the
// cycle is recorded once per starting state and replayed. Returns the relative residual.
int run_cycle(mg_ctx* m, const double* b, double* x, bool reuse, double* rel, hipStream_t s) {
  int st;
  if (!m->use_graphs || m->cycles_run == 0) {
    if ((st = enqueue_cycle(m, b, x, reuse, s)) != GABP_OK) return st;
  } else {
    const std::vector<int> before = parities(m);
    MgGraph* g = nullptr;
    for (auto& e : m->graphs)
      if (e.b == b && e.x == x && e.reuse == reuse && e.before == before) g = &e;
    if (!g) {
      if (m->graphs.size() >= 4) {
        (void)hipGraphExecDestroy(m->graphs.front().exec);
        m->graphs.erase(m->graphs.begin());
      }
      if (!m->capture_stream)
        GABP_HIP(hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking));
      GABP_HIP(hipStreamBeginCapture(m->capture_stream, hipStreamCaptureModeThreadLocal));
      st = enqueue_cycle(m, b, x, reuse, m->capture_stream);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(m->capture_stream, &graph);
      if (st != GABP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        set_parities(m, before);
        return st;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture (V-cycle)");
      MgGraph ng;
      ng.b = b;
      ng.x = x;
      ng.reuse = reuse;
      ng.before = before;
      ng.after = parities(m);
      const hipError_t e2 = hipGraphInstantiate(&ng.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate (V-cycle)");
      m->graphs.push_back(ng);
      g = &m->graphs.back();
    }
    GABP_HIP(hipGraphLaunch(g->exec, s));
    set_parities(m, g->after);
  }
  ++m->cycles_run;
  GABP_HIP(hipStreamSynchronize(s));
  const double* h = m->lv[0]->host_red;
  const double r2 = std::sqrt(h[0]), b2 = std::sqrt(h[2]);
  *rel = b2 > 0 ? r2 / b2 : r2;
  return GABP_OK;
}

}  // namespace

extern "C" {

int mg_setup(mg_ctx** out, int32_t levels, gabp_ctx* const* level_ctx, const int32_t* side,
             int32_t smoother, int32_t nu1, int32_t nu2, hipStream_t s) {
  if (!out || !level_ctx || !side) return fail(GABP_EINVAL, "NULL argument");
  *out = nullptr;
  if (levels < 2) return fail(GABP_EINVAL, "multigrid needs at least two levels");
  if ((smoother != 0 && smoother != 1) || nu1 < 0 || nu2 < 0)
    return fail(GABP_EINVAL, "smoother must be 0 (GaBP) or 1 (red-black Gauss-Seidel), nu >= 0");
  for (int l = 0; l < levels; ++l) {
    if (!level_ctx[l]) return fail(GABP_EINVAL, "NULL level context");
    if (side[l] < 1 || static_cast<int64_t>(side[l]) * side[l] != level_ctx[l]->L.n)
      return fail(GABP_EINVAL, "level " + std::to_string(l) + ": n != side^2");
    if (l + 1 < levels && side[l] != 2 * side[l + 1] + 1)
      return fail(GABP_EINVAL, "level sides must satisfy n_l = 2 n_{l+1} + 1");
  }
  if (side[levels - 1] > 63) return fail(GABP_ENOTSUPP, "coarsest grid above 63 x 63");
  mg_ctx* m = new mg_ctx();
  m->levels = levels;
  for (int l = 0; l < levels; ++l) m->use_graphs = m->use_graphs && level_ctx[l]->opt.use_graphs;
  m->lv.assign(level_ctx, level_ctx + levels);
  m->side.assign(side, side + levels);
  m->smoother = smoother;
  m->nu1 = nu1;
  m->nu2 = nu2;
  m->b.assign(levels, nullptr);
  m->x.assign(levels, nullptr);
  m->r.assign(levels, nullptr);
  auto bail = [&](int code) {
    mg_destroy(m);
    return code;
  };
  for (int l = 0; l < levels; ++l) {
    const size_t bytes = static_cast<size_t>(level_ctx[l]->L.n) * sizeof(double);
    if (hipMalloc(reinterpret_cast<void**>(&m->r[l]), bytes) != hipSuccess) return bail(fail(GABP_ENOMEM, "mg buffers"));
    if (l > 0) {
      if (hipMalloc(reinterpret_cast<void**>(&m->b[l]), bytes) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&m->x[l]), bytes) != hipSuccess)
        return bail(fail(GABP_ENOMEM, "mg buffers"));
    }
  }
  std::vector<double> A, inv;
  int st = dense_of(level_ctx[levels - 1], A, s);
  if (st != GABP_OK) return bail(st);
  m->nc = level_ctx[levels - 1]->L.n;
  if ((st = invert_dense(A, m->nc, inv)) != GABP_OK) return bail(st);
  if (hipMalloc(reinterpret_cast<void**>(&m->inv), inv.size() * sizeof(double)) != hipSuccess)
    return bail(fail(GABP_ENOMEM, "coarse inverse"));
  if (hipMemcpyAsync(m->inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(GABP_EDEVICE, "upload coarse inverse"));
  *out = m;
  return GABP_OK;
}

int mg_vcycle(mg_ctx* m, const double* b, double* x, double* rel_res_out, hipStream_t s) {
  if (!m || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  double rel = 0.0;
  const int st = run_cycle(m, b, x, false, &rel, s);   // x may have changed since
  if (st != GABP_OK) return st;
  if (rel_res_out) *rel_res_out = rel;
  return GABP_OK;
}

int mg_solve(mg_ctx* m, const double* b, double* x, double tol, int32_t max_cycles,
             int32_t* cycles_out, double* rel_res_out, hipStream_t s) {
  if (!m || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  if (max_cycles < 1) return fail(GABP_EINVAL, "max_cycles < 1");
  GABP_HIP(launch_fill64(x, m->lv[0]->L.n, 0.0, s));
  double rel = 1.0;
  int k = 0, st;
  while (k < max_cycles) {
    // from the second cycle on, x is the one the previous check's residual was formed for
    if ((st = run_cycle(m, b, x, k > 0, &rel, s)) != GABP_OK) return st;
    ++k;
    if (!std::isfinite(rel)) {
      if (cycles_out) *cycles_out = k;
      if (rel_res_out) *rel_res_out = rel;
      return fail(GABP_ENUMERIC, "multigrid diverged");
    }
    if (rel <= tol) break;
  }
  if (cycles_out) *cycles_out = k;
  if (rel_res_out) *rel_res_out = rel;
  return rel <= tol ? GABP_OK : GABP_MAXSWEEPS;
}

void mg_destroy(mg_ctx* m) {
  if (!m) return;
  for (auto& g : m->graphs) (void)hipGraphExecDestroy(g.exec);
  if (m->capture_stream) (void)hipStreamDestroy(m->capture_stream);
  for (double* p : m->b) if (p) (void)hipFree(p);
  for (double* p : m->x) if (p) (void)hipFree(p);
  for (double* p : m->r) if (p) (void)hipFree(p);
  if (m->inv) (void)hipFree(m->inv);
  delete m;
}

}  // extern "C"
