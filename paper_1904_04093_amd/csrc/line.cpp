// Host side of line GaBP (the two-layer region iteration on the rows and columns of a grid,
// Sec. 3 / Algorithm 2 with the partition of Fig. two_layers_network): the row and column
// layouts built from a 5-point grid matrix, the sweep drivers for the flood and the
// rows-then-columns schedules, the precision-message phase and the frozen multipliers.
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "gabp_line.h"

namespace gabp {
namespace {

template <typename T>
int dev_alloc(T** p, int64_t n) {
  GABP_HIP(hipMalloc(reinterpret_cast<void**>(p), (n > 0 ? n : 1) * sizeof(T)));
  return GABP_OK;
}

template <typename T>
int dev_upload(T** p, const std::vector<T>& h) {
  int st = dev_alloc(p, static_cast<int64_t>(h.size()));
  if (st != GABP_OK) return st;
  GABP_HIP(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return GABP_OK;
}

template <typename T>
int dev_zeros(T** p, int64_t n) {
  int st = dev_alloc(p, n);
  if (st != GABP_OK) return st;
  GABP_HIP(hipMemset(*p, 0, (n > 0 ? n : 1) * sizeof(T)));
  return GABP_OK;
}

std::vector<double> values_of(const std::vector<int32_t>& src, const double* val) {
  std::vector<double> v(src.size());
  for (size_t k = 0; k < src.size(); ++k) v[k] = src[k] >= 0 ? val[src[k]] : 0.0;
  return v;
}

// transpose jobs for the messages sent by one orientation (own layout -> other layout)
int transpose_side(const LineLayout& G, int o, bool lam, hipStream_t s) {
  const LineSide& S = G.side[o];
  const int rows = o == 0 ? G.ny : G.nx, cols = o == 0 ? G.nx : G.ny;
  TransposeJob<double> j[2];
  int nj = 0;
  if (lam) j[nj++] = TransposeJob<double>{S.lam_own, S.lam_x, rows, cols};
  j[nj++] = TransposeJob<double>{S.m_own, S.m_x, rows, cols};
  GABP_HIP(launch_transpose64(j, nj, s));
  return GABP_OK;
}

int transpose_side32(const LineLayout& G, int o, hipStream_t s) {
  const LineSide& S = G.side[o];
  const int rows = o == 0 ? G.ny : G.nx, cols = o == 0 ? G.nx : G.ny;
  TransposeJob<float> j{S.m32_own, S.m32_x, rows, cols};
  GABP_HIP(launch_transpose32(&j, 1, s));
  return GABP_OK;
}

// joint arguments of both orientations for transposition T and right-hand side b
void joint_args(const LineLayout& G, int T, const double* b_row, const double* b_col,
                LineArgs a[2]) {
  const LineSide& R = G.side[0];
  const LineSide& C = G.side[1];
  a[0] = LineArgs{R.nlines, R.len, R.diag, R.lo[T], R.hi[T], b_row, C.lam_x, C.m_x,
                  R.lam_own, R.m_own, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                  nullptr};
  a[1] = LineArgs{C.nlines, C.len, C.diag, C.lo[T], C.hi[T], b_col, R.lam_x, R.m_x,
                  C.lam_own, C.m_own, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                  nullptr};
}

// Read-off of the column update just made (before the column messages move to the row
// layout): x = (b + m_row + m_col) / (A_ii + Lambda_row + Lambda_col) in the column layout
// with the row messages that update used (flood: previous sweep, zero when rows_zero; alt:
// this sweep), then transposed into x (row layout). invS: frozen 1/Sigma* in the column
// layout, or null.
int readoff_col64(const LineLayout& G, const double* invS, double* x, hipStream_t s,
                  bool rows_zero = false) {
  const LineSide& R = G.side[0];
  const LineSide& C = G.side[1];
  GABP_HIP(launch_line_readoff64(G.n, G.bcol, C.diag, rows_zero ? nullptr : R.lam_x,
                                 rows_zero ? nullptr : R.m_x, C.lam_own, C.m_own, invS,
                                 G.xcol, s));
  TransposeJob<double> j{G.xcol, x, G.nx, G.ny};
  GABP_HIP(launch_transpose64(&j, 1, s));
  return GABP_OK;
}

// one joint update of every line (flood: both orientations from the previous messages;
// alt: rows, then columns from the new row messages); x != null: the read-off. first: the
// update right after a reset (the incoming arrays of a are null where the messages are zero)
int joint_update(const LineLayout& G, LineArgs a[2], double* x, hipStream_t s,
                 bool first = false) {
  int st;
  if (!G.alt) {
    GABP_HIP(launch_line_joint(a, 2, s));
    if (x && (st = readoff_col64(G, nullptr, x, s, first)) != GABP_OK) return st;
    if ((st = transpose_side(G, 0, true, s)) != GABP_OK) return st;
    return transpose_side(G, 1, true, s);
  }
  for (int o = 0; o < 2; ++o) {
    GABP_HIP(launch_line_joint(&a[o], 1, s));
    if (o == 1 && x && (st = readoff_col64(G, nullptr, x, s)) != GABP_OK) return st;
    if ((st = transpose_side(G, o, true, s)) != GABP_OK) return st;
  }
  return GABP_OK;
}

int zero_joint(const LineLayout& G, hipStream_t s) {
  for (int o = 0; o < 2; ++o) {
    const LineSide& S = G.side[o];
    GABP_HIP(launch_fill64(S.lam_own, G.n, 0.0, s));
    GABP_HIP(launch_fill64(S.lam_x, G.n, 0.0, s));
    GABP_HIP(launch_fill64(S.m_own, G.n, 0.0, s));
    GABP_HIP(launch_fill64(S.m_x, G.n, 0.0, s));
  }
  return GABP_OK;
}

}  // namespace

int line_setup(gabp_ctx* c, int nx, int ny, const int32_t* rowptr, const int32_t* col,
               const double* val) {
  const int64_t n = c->L.n;
  if (nx < 1 || ny < 1 || static_cast<int64_t>(nx) * ny != n)
    return fail(GABP_EINVAL, "line schedules need grid_nx * grid_ny == n");
  if (nx > kLineMaxLen || ny > kLineMaxLen)
    return fail(GABP_ENOTSUPP, "line GaBP supports lines of at most " +
                                   std::to_string(kLineMaxLen) + " nodes");
  // CSR index of the diagonal and of the W, E, S, N couplings of every node
  std::vector<int32_t> iD(n, -1), iW(n, -1), iE(n, -1), iS(n, -1), iN(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t x = i % nx;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int64_t j = col[e];
      if (j == i) iD[i] = static_cast<int32_t>(e);
      else if (j == i - 1 && x > 0) iW[i] = static_cast<int32_t>(e);
      else if (j == i + 1 && x < nx - 1) iE[i] = static_cast<int32_t>(e);
      else if (j == i - nx) iS[i] = static_cast<int32_t>(e);
      else if (j == i + nx) iN[i] = static_cast<int32_t>(e);
      else
        return fail(GABP_EINVAL, "entry (" + std::to_string(i) + ", " + std::to_string(j) +
                                     ") does not join grid neighbours: line GaBP needs a "
                                     "5-point grid operator");
    }
  }
  auto* G = new LineLayout();
  c->lines = G;
  G->nx = nx;
  G->ny = ny;
  G->n = n;
  G->alt = c->opt.schedule == GABP_SCHED_LINES_ALT;
  {
    constexpr double kLLC = 256.0 * 1024 * 1024;   // last-level cache
    G->nt64 = 40.0 * 2 * static_cast<double>(n) > kLLC;
    G->nt32 = 20.0 * 2 * static_cast<double>(n) > kLLC;
  }
  // side 0: rows, index y*nx + x, predecessor W, successor E
  // side 1: columns, index x*ny + y, predecessor S, successor N
  // A^T along a line: (A^T)_{t,t-1} = A_{t-1,t} (successor coupling of t-1) and
  // (A^T)_{t,t+1} = A_{t+1,t} (predecessor coupling of t+1)
  for (int o = 0; o < 2; ++o) {
    LineSide& S = G->side[o];
    S.nlines = o == 0 ? ny : nx;
    S.len = o == 0 ? nx : ny;
    std::vector<int32_t> d(n), lo0(n), hi0(n), lo1(n, -1), hi1(n, -1);
    for (int64_t line = 0; line < S.nlines; ++line)
      for (int64_t t = 0; t < S.len; ++t) {
        const int64_t k = line * S.len + t;
        const int64_t i = o == 0 ? line * nx + t : t * nx + line;   // grid node
        d[k] = iD[i];
        lo0[k] = o == 0 ? iW[i] : iS[i];
        hi0[k] = o == 0 ? iE[i] : iN[i];
      }
    for (int64_t line = 0; line < S.nlines; ++line)
      for (int64_t t = 0; t < S.len; ++t) {
        const int64_t k = line * S.len + t;
        if (t > 0) lo1[k] = hi0[k - 1];
        if (t + 1 < S.len) hi1[k] = lo0[k + 1];
      }
    int st;
    if ((st = dev_upload(&S.diag, values_of(d, val))) || (st = dev_upload(&S.lo[0], values_of(lo0, val))) ||
        (st = dev_upload(&S.hi[0], values_of(hi0, val))) || (st = dev_upload(&S.lo[1], values_of(lo1, val))) ||
        (st = dev_upload(&S.hi[1], values_of(hi1, val))) || (st = dev_upload(&S.diag_src, d)) ||
        (st = dev_upload(&S.lo_src[0], lo0)) || (st = dev_upload(&S.hi_src[0], hi0)) ||
        (st = dev_upload(&S.lo_src[1], lo1)) || (st = dev_upload(&S.hi_src[1], hi1)) ||
        (st = dev_zeros(&S.lam_own, n)) || (st = dev_zeros(&S.m_own, n)) ||
        (st = dev_zeros(&S.lam_x, n)) || (st = dev_zeros(&S.m_x, n)))
      return st;
  }
  int st;
  if ((st = dev_zeros(&G->bcol, n)) || (st = dev_zeros(&G->zero, n)) ||
      (st = dev_zeros(&G->xcol, n)) ||
      (st = dev_zeros(&G->partials, 2 * static_cast<int64_t>(nx + ny))))
    return st;
  return GABP_OK;
}

void line_destroy(LineLayout* G) {
  if (!G) return;
  auto F = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto& S : G->side) {
    F(S.diag); F(S.diag_src); F(S.lam_own); F(S.m_own); F(S.lam_x); F(S.m_x);
    F(S.m32_own); F(S.m32_x);
    for (int T = 0; T < 2; ++T) {
      F(S.lo[T]); F(S.hi[T]); F(S.lo_src[T]); F(S.hi_src[T]);
      F(S.alpha[T]); F(S.beta[T]); F(S.alpha32[T]); F(S.beta32[T]);
    }
  }
  F(G->bcol); F(G->bcol32); F(G->zero); F(G->partials); F(G->xcol); F(G->xcol32);
  for (int T = 0; T < 2; ++T) {
    F(G->invS[T]); F(G->invS32[T]);
  }
  delete G;
}

int line_update_values(gabp_ctx* c, const double* val, hipStream_t s) {
  LineLayout& G = *c->lines;
  for (auto& S : G.side) {
    GABP_HIP(launch_gather_values(G.n, S.diag_src, val, S.diag, s));
    for (int T = 0; T < 2; ++T) {
      GABP_HIP(launch_gather_values(G.n, S.lo_src[T], val, S.lo[T], s));
      GABP_HIP(launch_gather_values(G.n, S.hi_src[T], val, S.hi[T], s));
    }
  }
  return GABP_OK;
}

// Zero messages. Only the incoming copies a sweep reads before anything writes them are
// zero -- the column messages in the row layout, and (flood) the row messages in the column
// layout; the rows-then-columns schedule rewrites the latter before the columns read them,
// and every outgoing array is written by its own update before anything reads it. With
// precomputed Lambda only the mean messages restart. A reset only marks them (c->fresh64):
// the next sweep passes null for them; line_zero_incoming64 writes the zeros out when
// the arrays themselves are needed (checkpoints, fault injection).
int line_reset64(gabp_ctx* c, hipStream_t s) {
  (void)s;
  c->fresh64 = true;
  return GABP_OK;
}

int line_zero_incoming64(gabp_ctx* c, hipStream_t s) {
  if (!c->fresh64) return GABP_OK;
  const LineLayout& G = *c->lines;
  const bool joint = c->opt.mode == GABP_MODE_JOINT;
  for (int o = 1; o >= (G.alt ? 1 : 0); --o) {   // columns' messages (row layout), then rows'
    const LineSide& S = G.side[o];
    GABP_HIP(launch_fill64(S.m_x, G.n, 0.0, s));
    if (joint) GABP_HIP(launch_fill64(S.lam_x, G.n, 0.0, s));
  }
  c->fresh64 = false;
  return GABP_OK;
}

int line_ensure32(gabp_ctx* c, hipStream_t s) {
  LineLayout& G = *c->lines;
  if (G.side[0].m32_own) return GABP_OK;
  int st;
  for (auto& S : G.side)
    if ((st = dev_zeros(&S.m32_own, G.n)) || (st = dev_zeros(&S.m32_x, G.n))) return st;
  if ((st = dev_zeros(&G.bcol32, G.n)) || (st = dev_zeros(&G.xcol32, G.n))) return st;
  (void)s;
  return GABP_OK;
}

bool line_has32(const gabp_ctx* c) { return c->lines->side[0].m32_own != nullptr; }

int line_reset32(gabp_ctx* c, hipStream_t s) {   // as line_reset64
  (void)s;
  c->fresh32 = true;
  return GABP_OK;
}

int line_zero_incoming32(gabp_ctx* c, hipStream_t s) {
  if (!c->fresh32) return GABP_OK;
  const LineLayout& G = *c->lines;
  if (G.side[0].m32_x)
    for (int o = 1; o >= (G.alt ? 1 : 0); --o) GABP_HIP(launch_fill32(G.side[o].m32_x, G.n, 0.0f, s));
  c->fresh32 = false;
  return GABP_OK;
}

int line_rhs64(gabp_ctx* c, const double* b, hipStream_t s) {
  const LineLayout& G = *c->lines;
  TransposeJob<double> j{b, G.bcol, G.ny, G.nx};
  GABP_HIP(launch_transpose64(&j, 1, s));
  return GABP_OK;
}

int line_rhs32(gabp_ctx* c, const float* b, hipStream_t s) {
  const LineLayout& G = *c->lines;
  TransposeJob<float> j{b, G.bcol32, G.ny, G.nx};
  GABP_HIP(launch_transpose32(&j, 1, s));
  return GABP_OK;
}

// GABP_FAULT_INJECT=poison-outputs: NaN into the arrays a line update only writes (the
// messages in the sender's own layout) before the update.
static int poison_own(gabp_ctx* c, bool f32, hipStream_t s) {
  if (!c->poison_outputs) return GABP_OK;
  const LineLayout& G = *c->lines;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (const auto& S : G.side) {
    if (f32) {
      GABP_HIP(launch_fill32(S.m32_own, G.n, static_cast<float>(nan), s));
      continue;
    }
    GABP_HIP(launch_fill64(S.m_own, G.n, nan, s));
    if (c->opt.mode != GABP_MODE_PRECOMP) GABP_HIP(launch_fill64(S.lam_own, G.n, nan, s));
  }
  return GABP_OK;
}

int line_sweep64(gabp_ctx* c, int T, const double* b, double* x, hipStream_t s) {
  const LineLayout& G = *c->lines;
  const LineSide& R = G.side[0];
  const LineSide& C = G.side[1];
  int st;
  if ((st = poison_own(c, false, s)) != GABP_OK) return st;
  // first sweep after a reset: the columns' messages (and for flood the rows') are zero
  const bool first = c->fresh64;
  c->fresh64 = false;
  const bool rows_zero = first && !G.alt;
  if (c->opt.mode != GABP_MODE_PRECOMP) {
    LineArgs a[2];
    joint_args(G, T, b, G.bcol, a);
    if (first) a[0].lam_in = a[0].m_in = nullptr;
    if (rows_zero) a[1].lam_in = a[1].m_in = nullptr;
    return joint_update(G, a, x, s, first);
  }
  LineMeanArgs<double> m[2] = {
      {R.nlines, R.len, R.alpha[T], R.beta[T], b, first ? nullptr : C.m_x, R.m_own, G.nt64},
      {C.nlines, C.len, C.alpha[T], C.beta[T], G.bcol, rows_zero ? nullptr : R.m_x, C.m_own,
       G.nt64}};
  if (!G.alt) {
    GABP_HIP(launch_line_mean64(m, 2, s));
    if (x && (st = readoff_col64(G, G.invS[T], x, s, rows_zero)) != GABP_OK) return st;
    if ((st = transpose_side(G, 0, false, s)) != GABP_OK) return st;
    return transpose_side(G, 1, false, s);
  }
  for (int o = 0; o < 2; ++o) {
    GABP_HIP(launch_line_mean64(&m[o], 1, s));
    if (o == 1 && x && (st = readoff_col64(G, G.invS[T], x, s)) != GABP_OK) return st;
    if ((st = transpose_side(G, o, false, s)) != GABP_OK) return st;
  }
  return GABP_OK;
}

int line_sweep32(gabp_ctx* c, int T, const float* b, float* x, hipStream_t s) {
  const LineLayout& G = *c->lines;
  const LineSide& R = G.side[0];
  const LineSide& C = G.side[1];
  int st;
  if ((st = poison_own(c, true, s)) != GABP_OK) return st;
  const bool first = c->fresh32;   // as line_sweep64
  c->fresh32 = false;
  const bool rows_zero = first && !G.alt;
  auto readoff = [&]() -> int {
    GABP_HIP(launch_line_readoff32(G.n, G.bcol32, rows_zero ? nullptr : R.m32_x, C.m32_own,
                                   G.invS32[T], G.xcol32, s));
    TransposeJob<float> j{G.xcol32, x, G.nx, G.ny};
    GABP_HIP(launch_transpose32(&j, 1, s));
    return GABP_OK;
  };
  LineMeanArgs<float> m[2] = {
      {R.nlines, R.len, R.alpha32[T], R.beta32[T], b, first ? nullptr : C.m32_x, R.m32_own,
       G.nt32},
      {C.nlines, C.len, C.alpha32[T], C.beta32[T], G.bcol32, rows_zero ? nullptr : R.m32_x,
       C.m32_own, G.nt32}};
  if (!G.alt) {
    GABP_HIP(launch_line_mean32(m, 2, s));
    if (x && (st = readoff()) != GABP_OK) return st;
    if ((st = transpose_side32(G, 0, s)) != GABP_OK) return st;
    return transpose_side32(G, 1, s);
  }
  for (int o = 0; o < 2; ++o) {
    GABP_HIP(launch_line_mean32(&m[o], 1, s));
    if (o == 1 && x && (st = readoff()) != GABP_OK) return st;
    if ((st = transpose_side32(G, o, s)) != GABP_OK) return st;
  }
  return GABP_OK;
}

static int alloc_pre(LineLayout& G, int T) {
  int st;
  for (auto& S : G.side)
    if (!S.alpha[T] &&
        ((st = dev_alloc(&S.alpha[T], G.n)) || (st = dev_alloc(&S.beta[T], G.n)) ||
         (st = dev_alloc(&S.alpha32[T], G.n)) || (st = dev_alloc(&S.beta32[T], G.n))))
      return st;
  if (!G.invS[T] && ((st = dev_alloc(&G.invS[T], G.n)) || (st = dev_alloc(&G.invS32[T], G.n))))
    return st;
  return GABP_OK;
}

int line_state_arrays(gabp_ctx* c, bool has32, const bool pre[2], bool alloc,
                      std::vector<StateArray>* out) {
  LineLayout& G = *c->lines;
  const size_t n = static_cast<size_t>(G.n);
  int st;
  out->clear();
  for (auto& S : G.side)
    for (double* p : {S.lam_own, S.m_own, S.lam_x, S.m_x}) out->push_back({p, n * sizeof(double)});
  if (has32) {
    if (alloc && (st = line_ensure32(c, nullptr)) != GABP_OK) return st;
    for (auto& S : G.side)
      for (float* p : {S.m32_own, S.m32_x}) out->push_back({p, n * sizeof(float)});
  }
  for (int T = 0; T < 2; ++T) {
    if (!pre[T]) continue;
    if (alloc && (st = alloc_pre(G, T)) != GABP_OK) return st;
    for (auto& S : G.side) {
      out->push_back({S.alpha[T], n * sizeof(double)});
      out->push_back({S.beta[T], n * sizeof(double)});
      out->push_back({S.alpha32[T], n * sizeof(float)});
      out->push_back({S.beta32[T], n * sizeof(float)});
    }
    out->push_back({G.invS[T], n * sizeof(double)});
    out->push_back({G.invS32[T], n * sizeof(float)});
  }
  for (const auto& a : *out)
    if (!a.p) return fail(GABP_EINVAL, "line state array missing");
  return GABP_OK;
}

// Precision phase: iterate the Lambda messages alone (zero right-hand side, so the mean
// messages stay zero) until max|dLambda| <= tol_lambda * max|Lambda|, then the frozen
// multipliers alpha, beta from the final messages and 1/Sigma* for the read-off.
int line_precompute(gabp_ctx* c, int T, hipStream_t s) {
  Precomp& P = c->pre[T];
  if (P.valid) return GABP_OK;
  LineLayout& G = *c->lines;
  int st;
  if ((st = alloc_pre(G, T)) != GABP_OK) return st;
  if ((st = zero_joint(G, s)) != GABP_OK) return st;
  const LineSide& R = G.side[0];
  const LineSide& C = G.side[1];
  LineArgs a[2];
  joint_args(G, T, G.zero, G.zero, a);
  a[0].partials = G.partials;
  a[1].partials = G.alt ? G.partials + 2 * static_cast<int64_t>(R.nlines) : G.partials;
  const double tol = c->opt.tol_lambda;
  int done = 0;
  for (int it = 1; it <= c->opt.max_lambda_sweeps; ++it) {
    if ((st = joint_update(G, a, nullptr, s)) != GABP_OK) return st;
    GABP_HIP(launch_max_pairs(R.nlines + C.nlines, G.partials, c->red + 5, s));
    done = it;
    if (tol > 0.0) {
      GABP_HIP(hipMemcpyAsync(c->host_red + 5, c->red + 5, 2 * sizeof(double),
                              hipMemcpyDeviceToHost, s));
      GABP_HIP(hipStreamSynchronize(s));
      const double dm = c->host_red[5], lm = c->host_red[6];
      if (!std::isfinite(dm) || !std::isfinite(lm))
        return fail(GABP_ENUMERIC, "non-finite precision message in the Lambda phase");
      if (dm <= tol * lm) break;
    }
  }
  // frozen multipliers from the final messages (both orientations, one launch), and the
  // read-off factor of the frozen column systems, 1 / (T^{-1})_tt, in the column layout
  LineArgs f[2];
  joint_args(G, T, G.zero, G.zero, f);
  for (int o = 0; o < 2; ++o) {
    LineSide& S = G.side[o];
    f[o].lam_out = nullptr;
    f[o].m_out = nullptr;
    f[o].alpha = S.alpha[T];
    f[o].beta = S.beta[T];
    f[o].alpha32 = S.alpha32[T];
    f[o].beta32 = S.beta32[T];
  }
  f[1].invS = G.invS[T];
  f[1].invS32 = G.invS32[T];
  GABP_HIP(launch_line_joint(f, 2, s));
  if ((st = zero_joint(G, s)) != GABP_OK) return st;
  P.sweeps = done;
  P.valid = true;
  return GABP_OK;
}

}  // namespace gabp
