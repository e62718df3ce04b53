// Solve drivers of libgabp: Algorithm 1 in the flood (or red-black) schedule, the
// precomputed-Lt variant, FP32-message iterative refinement, the error-correction smoother
// (Algorithm 3), residuals, the adjoint scatter and checkpoints.
//
// All device work is enqueued on the caller's stream. Convergence is read back every
// `check_every` sweeps through one small pinned buffer; nothing else synchronises.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "gabp_internal.h"
#include "gabp_line.h"
#include "graph.h"

using namespace gabp;

namespace gabp {

void free_seq(gabp_ctx* c) {
  SeqPrecomp& Q = c->seq;
  for (double* p : Q.lamout) (void)hipFree(p);
  for (double* p : Q.S) (void)hipFree(p);
  for (float* p : Q.lamout32) (void)hipFree(p);
  for (float* p : Q.invS32) (void)hipFree(p);
  Q = SeqPrecomp{};
}

// Lt-only sweeps from zero messages in the context's schedule, keeping what each sweep
// computes. Entries already allocated keep their addresses (recorded graphs read them in
// place); the joint-mode Lt buffers, unused in this mode, hold the running Lt state.
int ensure_seq(gabp_ctx* c, int depth, hipStream_t s) {
  SeqPrecomp& Q = c->seq;
  if (Q.valid && Q.depth >= depth) return GABP_OK;
  depth = std::max(depth, Q.depth);
  const Layout& L = c->L;
  const int64_t E = L.epad + 1;
  while (static_cast<int>(Q.lamout.size()) < depth) {
    double* d = nullptr;
    float* f = nullptr;
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&d), E * sizeof(double)));
    Q.lamout.push_back(d);
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&d), L.n * sizeof(double)));
    Q.S.push_back(d);
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&f), E * sizeof(float)));
    Q.lamout32.push_back(f);
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&f), L.n * sizeof(float)));
    Q.invS32.push_back(f);
  }
  GABP_HIP(launch_fill64(c->lam[0], E, 0.0, s));
  GABP_HIP(launch_fill64(c->lam[1], E, 0.0, s));
  const bool coloured = c->opt.schedule == GABP_SCHED_REDBLACK;
  int par = 0;
  for (int k = 0; k < depth; ++k) {
    if (coloured) {
      for (int col = 0; col < L.ncolours; ++col)
        GABP_HIP(launch_lambda_step(&L, L.aT, c->lam[0], c->lam[0], Q.lamout[k], Q.lamout32[k],
                                    Q.S[k], Q.invS32[k], col, s));
    } else {
      GABP_HIP(launch_lambda_step(&L, L.aT, c->lam[par], c->lam[par ^ 1], Q.lamout[k],
                                  Q.lamout32[k], Q.S[k], Q.invS32[k], -1, s));
      par ^= 1;
    }
  }
  Q.depth = depth;
  Q.valid = true;
  return GABP_OK;
}

}  // namespace gabp

namespace {

inline bool seq_mode(const gabp_ctx* c) { return c->opt.mode == GABP_MODE_PRECOMP_SEQ; }

// Progress lines of long solves (opt.progress_s > 0), printed from the solve's own checks.
struct Progress {
  using Clock = std::chrono::steady_clock;
  double every;
  Clock::time_point t0, last;
  explicit Progress(double e) : every(e), t0(Clock::now()), last(t0) {}
  void check(int sweeps, int outer, double rel) {
    if (every <= 0.0) return;
    const auto now = Clock::now();
    if (std::chrono::duration<double>(now - last).count() < every) return;
    last = now;
    std::fprintf(stderr, "[gabp] %d sweeps, %d refinement steps, rel.res %.3e, %.0f s\n",
                 sweeps, outer, rel, std::chrono::duration<double>(now - t0).count());
    std::fflush(stderr);
  }
};

struct Norms {
  double r2, rinf, b2;
};

void host_norms(const gabp_ctx* c, Norms* nm) {
  nm->r2 = std::sqrt(c->host_red[0]);
  nm->rinf = c->host_red[1];
  nm->b2 = std::sqrt(c->host_red[2]);
}

int read_norms(gabp_ctx* c, hipStream_t s, Norms* nm) {
  GABP_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  GABP_HIP(hipStreamSynchronize(s));
  nm->r2 = std::sqrt(c->host_red[0]);
  nm->rinf = c->host_red[1];
  nm->b2 = std::sqrt(c->host_red[2]);
  return GABP_OK;
}

inline const double* sweep_coef(const gabp_ctx* c, int T) { return T ? c->L.val : c->L.aT; }
inline const double* row_coef(const gabp_ctx* c, int T) { return T ? c->L.aT : c->L.val; }

int residual(gabp_ctx* c, int T, const double* b, const double* x, const float* dx,
             const double* scale, double* r, hipStream_t s, bool norms = true,
             float* r32 = nullptr) {
  GABP_HIP(launch_residual(&c->L, row_coef(c, T), b, x, dx, scale, r, c->partials, c->nred,
                           c->red, s, norms, r32));
  return GABP_OK;
}

int ensure_pre(gabp_ctx* c, int T, hipStream_t s) {
  if (c->lines) return line_precompute(c, T, s);
  Precomp& P = c->pre[T];
  if (P.valid) return GABP_OK;
  const Layout& L = c->L;
  if (!P.lamout) {
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.lamout), (L.epad + 1) * sizeof(double)));
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.S), L.n * sizeof(double)));
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.lamout32), (L.epad + 1) * sizeof(float)));
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.invS32), L.n * sizeof(float)));
  }
  GABP_HIP(launch_fill64(P.lamout, L.epad + 1, 0.0, s));
  GABP_HIP(launch_fill64(c->lam[0], L.epad + 1, 0.0, s));
  GABP_HIP(launch_fill64(c->lam[1], L.epad + 1, 0.0, s));
  const double* coef = sweep_coef(c, T);
  if (2 * ((L.nlanes + kBlock - 1) / kBlock) > c->npartials)   // k_lambda's partials
    return fail(GABP_EINVAL, "internal: partials buffer smaller than the Lt phase needs");
  int par = 0, done = 0;
  const double tol = c->opt.tol_lambda;
  for (int it = 1; it <= c->opt.max_lambda_sweeps; ++it) {
    GABP_HIP(launch_lambda_sweep(&L, coef, c->lam[par], c->lam[par ^ 1], P.lamout, c->partials,
                                 c->red + 5, s));
    par ^= 1;
    done = it;
    if (tol > 0.0) {
      GABP_HIP(hipMemcpyAsync(c->host_red + 5, c->red + 5, 2 * sizeof(double),
                              hipMemcpyDeviceToHost, s));
      GABP_HIP(hipStreamSynchronize(s));
      const double dm = c->host_red[5], lm = c->host_red[6];
      if (!std::isfinite(dm) || !std::isfinite(lm))
        return fail(GABP_ENUMERIC, "non-finite precision message in the Lt phase");
      if (dm <= tol * lm) break;
    }
  }
  GABP_HIP(launch_lambda_finalize(&L, coef, c->lam[par], &P, s));
  P.sweeps = done;
  P.valid = true;
  c->parity = 0;   // the joint-mode message buffers were used as scratch: logically zero now
  c->fresh64 = true;
  return GABP_OK;
}

// Both FP32 message buffers start at zero: padding slots (short rows inside a slice) are
// read by every sweep but never written, so they must hold zeros in both buffers.
int ensure_msg32(gabp_ctx* c, hipStream_t s) {
  if (c->lines) {
    if (!c->dbest32) GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->dbest32), c->L.n * sizeof(float)));
    return line_ensure32(c, s);
  }
  if (c->msg32[0]) return GABP_OK;
  for (int q = 0; q < 2; ++q) {
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->msg32[q]), (c->L.epad + 1) * sizeof(float)));
    GABP_HIP(launch_fill32(c->msg32[q], c->L.epad + 1, 0.0f, s));
  }
  GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->dbest32), c->L.n * sizeof(float)));
  return GABP_OK;
}

// (the slot one past the padded slots holds no message and is left alone)
constexpr double kPoison = std::numeric_limits<double>::quiet_NaN();

// One FP64 sweep of the configured mode and schedule on right-hand side b (coloured
// schedule: the colour classes 0, 1, ... in turn, in place).
// x != null: the read-off of this sweep is written there; xadd != null instead: the
// read-off is added to xadd (xset: stored into it).
int sweep64(gabp_ctx* c, int T, const double* b, double* x, hipStream_t s,
            double* xadd = nullptr, bool xset = false) {
  if (c->lines) {
    if (!xadd) return line_sweep64(c, T, b, x, s);
    const int st = line_sweep64(c, T, b, c->e, s);
    if (st != GABP_OK) return st;
    GABP_HIP(xset ? launch_copy64(xadd, c->e, c->L.n, s) : launch_axpy64(xadd, c->e, c->L.n, s));
    return GABP_OK;
  }
  const bool rb = c->opt.schedule == GABP_SCHED_REDBLACK;
  const int fresh = c->fresh64 ? 0 : -1;   // first sweep after a reset
  c->fresh64 = false;
  if (c->opt.mode == GABP_MODE_JOINT) {
    SweepArgs a{&c->L, sweep_coef(c, T), b, nullptr, nullptr, nullptr, nullptr, x, -1, fresh};
    a.xadd = xadd;
    a.xset = xset;
    if (!rb) {
      a.lam_in = c->lam[c->parity];
      a.msg_in = c->msg[c->parity];
      a.lam_out = c->lam[c->parity ^ 1];
      a.msg_out = c->msg[c->parity ^ 1];
      if (c->poison_outputs) {
        GABP_HIP(launch_fill64(a.lam_out, c->L.epad, kPoison, s));
        GABP_HIP(launch_fill64(a.msg_out, c->L.epad, kPoison, s));
      }
      GABP_HIP(launch_joint_sweep(a, s));
      c->parity ^= 1;
    } else {
      a.lam_in = a.lam_out = c->lam[c->parity];
      a.msg_in = a.msg_out = c->msg[c->parity];
      for (int col = 0; col < c->L.ncolours; ++col) {
        a.colour = col;
        if (fresh >= 0) a.fresh = c->L.cslot[col];
        GABP_HIP(launch_joint_sweep(a, s));
      }
    }
  } else {
    const double* lo = c->pre[T].lamout;
    const double* Sx = c->pre[T].S;
    if (seq_mode(c)) {   // sweep seq_pos64 + 1 after the reset
      if (T != 0 || c->seq_pos64 >= c->seq.depth)
        return fail(GABP_EINVAL, "per-sweep precision messages missing for this sweep");
      lo = c->seq.lamout[c->seq_pos64];
      Sx = c->seq.S[c->seq_pos64];
      ++c->seq_pos64;
    }
    MeanArgs64 a{&c->L, lo, Sx, b, nullptr, nullptr, x, -1, fresh};
    a.xadd = xadd;
    a.xset = xset;
    if (!rb) {
      a.msg_in = c->msg[c->parity];
      a.msg_out = c->msg[c->parity ^ 1];
      if (c->poison_outputs) GABP_HIP(launch_fill64(a.msg_out, c->L.epad, kPoison, s));
      GABP_HIP(launch_mean_sweep64(a, s));
      c->parity ^= 1;
    } else {
      a.msg_in = a.msg_out = c->msg[c->parity];
      for (int col = 0; col < c->L.ncolours; ++col) {
        a.colour = col;
        if (fresh >= 0) a.fresh = c->L.cslot[col];
        GABP_HIP(launch_mean_sweep64(a, s));
      }
    }
  }
  return GABP_OK;
}

int sweep32(gabp_ctx* c, int T, const float* b, float* x, hipStream_t s,
            double* xadd = nullptr, bool xset = false) {
  if (c->lines) {
    if (!xadd) return line_sweep32(c, T, b, x, s);
    const int st = line_sweep32(c, T, b, c->d32, s);
    if (st != GABP_OK) return st;
    if (xset) GABP_HIP(launch_fill64(xadd, c->L.n, 0.0, s));
    GABP_HIP(launch_axpy32(xadd, c->d32, nullptr, c->L.n, s));
    return GABP_OK;
  }
  const float* lo = c->pre[T].lamout32;
  const float* iS = c->pre[T].invS32;
  if (seq_mode(c)) {
    if (T != 0 || c->seq_pos32 >= c->seq.depth)
      return fail(GABP_EINVAL, "per-sweep precision messages missing for this sweep");
    lo = c->seq.lamout32[c->seq_pos32];
    iS = c->seq.invS32[c->seq_pos32];
    ++c->seq_pos32;
  }
  const int fresh = c->fresh32 ? 0 : -1;   // first sweep after a reset
  c->fresh32 = false;
  MeanArgs32 a{&c->L, lo, iS, b, nullptr, nullptr, x, -1, fresh};
  a.xadd = xadd;
  a.xset = xset;
  if (c->opt.schedule != GABP_SCHED_REDBLACK) {
    a.msg_in = c->msg32[c->parity32];
    a.msg_out = c->msg32[c->parity32 ^ 1];
    if (c->poison_outputs)
      GABP_HIP(launch_fill32(a.msg_out, c->L.epad, static_cast<float>(kPoison), s));
    GABP_HIP(launch_mean_sweep32(a, s));
    c->parity32 ^= 1;
  } else {
    a.msg_in = a.msg_out = c->msg32[c->parity32];
    for (int col = 0; col < c->L.ncolours; ++col) {
      a.colour = col;
      if (fresh >= 0) a.fresh = c->L.cslot[col];
      GABP_HIP(launch_mean_sweep32(a, s));
    }
  }
  return GABP_OK;
}

// Two FP64 sweeps in one launch on a tiled layout (flood only); read-off as in sweep64.
int sweep64_pair(gabp_ctx* c, int T, const double* b, double* x, hipStream_t s,
                 double* xadd = nullptr, bool xset = false) {
  const int fresh = c->fresh64 ? 0 : -1;
  c->fresh64 = false;
  if (c->opt.mode == GABP_MODE_JOINT) {
    SweepArgs a{&c->L, sweep_coef(c, T), b, c->lam[c->parity], c->msg[c->parity],
                c->lam[c->parity ^ 1], c->msg[c->parity ^ 1], x, -1, fresh};
    a.xadd = xadd;
    a.xset = xset;
    if (c->poison_outputs) {
      GABP_HIP(launch_fill64(a.lam_out, c->L.epad, kPoison, s));
      GABP_HIP(launch_fill64(a.msg_out, c->L.epad, kPoison, s));
    }
    GABP_HIP(launch_joint_pair(a, s));
  } else {
    MeanPairArgs<double> a{&c->L, c->pre[T].lamout, c->pre[T].lamout, c->pre[T].S, b,
                           c->msg[c->parity], c->msg[c->parity ^ 1], x, fresh};
    if (seq_mode(c)) {
      const int k = c->seq_pos64;
      if (T != 0 || k + 1 >= c->seq.depth)
        return fail(GABP_EINVAL, "per-sweep precision messages missing for this sweep");
      a.lamA = c->seq.lamout[k];
      a.lamB = c->seq.lamout[k + 1];
      a.SxB = c->seq.S[k + 1];
      c->seq_pos64 += 2;
    }
    a.xadd = xadd;
    a.xset = xset;
    if (c->poison_outputs) GABP_HIP(launch_fill64(a.msg_out, c->L.epad, kPoison, s));
    GABP_HIP(launch_mean_pair64(a, s));
  }
  c->parity ^= 1;
  return GABP_OK;
}

int sweep32_pair(gabp_ctx* c, int T, const float* b, float* x, hipStream_t s,
                 double* xadd = nullptr, bool xset = false) {
  MeanPairArgs<float> a{&c->L, c->pre[T].lamout32, c->pre[T].lamout32, c->pre[T].invS32, b,
                        c->msg32[c->parity32], c->msg32[c->parity32 ^ 1], x,
                        c->fresh32 ? 0 : -1};
  if (seq_mode(c)) {
    const int k = c->seq_pos32;
    if (T != 0 || k + 1 >= c->seq.depth)
      return fail(GABP_EINVAL, "per-sweep precision messages missing for this sweep");
    a.lamA = c->seq.lamout32[k];
    a.lamB = c->seq.lamout32[k + 1];
    a.SxB = c->seq.invS32[k + 1];
    c->seq_pos32 += 2;
  }
  c->fresh32 = false;
  a.xadd = xadd;
  a.xset = xset;
  if (c->poison_outputs)
    GABP_HIP(launch_fill32(a.msg_out, c->L.epad, static_cast<float>(kPoison), s));
  GABP_HIP(launch_mean_pair32(a, s));
  c->parity32 ^= 1;
  return GABP_OK;
}

inline bool tiled(const gabp_ctx* c) { return c->L.ntiles > 0 && !c->lines; }

// launches that k sweeps take: pairs on a tiled layout, one each otherwise (the ping-pong
// parity flips once per launch)
inline int sweep_launches(const gabp_ctx* c, int k) { return tiled(c) ? k / 2 + k % 2 : k; }

// k FP64 sweeps; the read-off of the last goes to x (or is added to / stored into xadd)
int run_sweeps64(gabp_ctx* c, int T, const double* b, int k, double* x, hipStream_t s,
                 double* xadd = nullptr, bool xset = false) {
  for (int i = 0; i < k;) {
    const int step = tiled(c) && k - i >= 2 ? 2 : 1;
    const bool last = i + step == k;
    const int st = step == 2 ? sweep64_pair(c, T, b, last ? x : nullptr, s, last ? xadd : nullptr, xset)
                             : sweep64(c, T, b, last ? x : nullptr, s, last ? xadd : nullptr, xset);
    if (st != GABP_OK) return st;
    i += step;
  }
  return GABP_OK;
}

int run_sweeps32(gabp_ctx* c, int T, const float* b, int k, float* x, hipStream_t s,
                 double* xadd = nullptr, bool xset = false) {
  for (int i = 0; i < k;) {
    const int step = tiled(c) && k - i >= 2 ? 2 : 1;
    const bool last = i + step == k;
    const int st = step == 2 ? sweep32_pair(c, T, b, last ? x : nullptr, s, last ? xadd : nullptr, xset)
                             : sweep32(c, T, b, last ? x : nullptr, s, last ? xadd : nullptr, xset);
    if (st != GABP_OK) return st;
    i += step;
  }
  return GABP_OK;
}

// Point schedules: no clearing; the next sweep reads the buffers as zero (fresh flags).
// With poison-outputs the buffers the next sweep reads from are filled with NaN instead, so
// a first sweep (flood, or a colour class in place) that read a stale slot would show it.
int reset_messages64(gabp_ctx* c, hipStream_t s) {
  c->parity = 0;
  c->seq_pos64 = 0;
  if (c->lines) return line_reset64(c, s);
  c->fresh64 = true;
  if (c->poison_outputs) {
    if (c->opt.mode == GABP_MODE_JOINT) GABP_HIP(launch_fill64(c->lam[0], c->L.epad, kPoison, s));
    GABP_HIP(launch_fill64(c->msg[0], c->L.epad, kPoison, s));
  }
  return GABP_OK;
}

int reset_messages32(gabp_ctx* c, hipStream_t s) {
  c->parity32 = 0;
  c->seq_pos32 = 0;
  if (c->lines) return line_reset32(c, s);
  c->fresh32 = true;
  if (c->poison_outputs && c->msg32[0])
    GABP_HIP(launch_fill32(c->msg32[0], c->L.epad, static_cast<float>(kPoison), s));
  return GABP_OK;
}

// Line schedules read the right-hand side in both the row and the column layout: these
// refresh the column copy (no-ops for point schedules).
int prep_rhs64(gabp_ctx* c, const double* b, hipStream_t s) {
  return c->lines ? line_rhs64(c, b, s) : GABP_OK;
}
int prep_rhs32(gabp_ctx* c, const float* b, hipStream_t s) {
  return c->lines ? line_rhs32(c, b, s) : GABP_OK;
}

// in-place schedules keep one message buffer (no ping-pong parity)
inline bool in_place(const gabp_ctx* c) {
  return c->opt.schedule == GABP_SCHED_REDBLACK || c->lines != nullptr;
}

bool has_msg32(const gabp_ctx* c) { return c->lines ? line_has32(c) : c->msg32[0] != nullptr; }

void fill_info(gabp_info* info, int status, int sweeps, int lsweeps, int outer,
               const Norms& nm) {
  if (!info) return;
  info->status = status;
  info->sweeps = sweeps;
  info->lambda_sweeps = lsweeps;
  info->outer_iters = outer;
  info->rel_res2 = nm.b2 > 0 ? nm.r2 / nm.b2 : nm.r2;
  info->res_inf = nm.rinf;
}

// Fault injection: NaN into every incoming mean message of the current sweep (FP64, or the
// FP32 inner messages of the refinement), once, when the solve reaches the chosen sweep.
static int maybe_inject(gabp_ctx* c, int done, bool f32, hipStream_t s) {
  if (c->inject_nan_at < 0 || done < c->inject_nan_at) return GABP_OK;
  c->inject_nan_at = -1;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  if (c->lines) {
    int st;
    if ((st = f32 ? line_zero_incoming32(c, s) : line_zero_incoming64(c, s)) != GABP_OK) return st;
    for (const auto& S : c->lines->side) {
      if (f32) GABP_HIP(launch_fill32(S.m32_x, c->lines->n, static_cast<float>(nan), s));
      else GABP_HIP(launch_fill64(S.m_x, c->lines->n, nan, s));
    }
    return GABP_OK;
  }
  // a logically zero (reset) state is made explicit first, so the next sweep reads the NaN
  if (f32) {
    c->fresh32 = false;
    GABP_HIP(launch_fill32(c->msg32[c->parity32], c->L.epad + 1, static_cast<float>(nan), s));
    return GABP_OK;
  }
  if (c->fresh64 && c->opt.mode == GABP_MODE_JOINT)
    GABP_HIP(launch_fill64(c->lam[c->parity], c->L.epad + 1, 0.0, s));
  c->fresh64 = false;
  GABP_HIP(launch_fill64(c->msg[c->parity], c->L.epad + 1, nan, s));
  return GABP_OK;
}

// Plain FP64 solve (JOINT or PRECOMP, flood or red-black).
int solve64(gabp_ctx* c, int T, const double* b, double* x, double tol, int max_sweeps,
            gabp_info* info, hipStream_t s) {
  int st, lsw = 0;
  if (c->opt.mode == GABP_MODE_PRECOMP) {
    const bool had = c->pre[T].valid;
    if ((st = ensure_pre(c, T, s)) != GABP_OK) return st;
    lsw = had ? 0 : c->pre[T].sweeps;
  }
  if ((st = reset_messages64(c, s)) != GABP_OK) return st;
  if ((st = prep_rhs64(c, b, s)) != GABP_OK) return st;
  Norms nm{0, 0, 0};
  int done = 0;
  const bool rb = in_place(c);
  c->history.clear();
  Progress prog(c->opt.progress_s);
  while (done < max_sweeps) {
    const int k = std::min(c->opt.check_every, max_sweeps - done);
    if ((st = maybe_inject(c, done, false, s)) != GABP_OK) return st;
    const int start = c->parity;
    const bool fresh = c->fresh64;
    // one check block: k sweeps (read-off on the last), residual, norms to the host
    st = run_block(c, *c->graphs, s, GraphKey{1, b, x, nullptr, start + 2 * fresh, k, T, 0.0},
                   [&](hipStream_t ss) -> int {
                     c->parity = start;
                     c->fresh64 = fresh;
                     int e = run_sweeps64(c, T, b, k, x, ss);
                     if (e != GABP_OK) return e;
                     e = residual(c, T, b, x, nullptr, nullptr, nullptr, ss);
                     if (e != GABP_OK) return e;
                     GABP_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double),
                                             hipMemcpyDeviceToHost, ss));
                     return GABP_OK;
                   });
    if (st != GABP_OK) return st;
    c->parity = rb ? start : start ^ (sweep_launches(c, k) & 1);
    c->fresh64 = false;
    done += k;
    GABP_HIP(hipStreamSynchronize(s));
    host_norms(c, &nm);
    const double rel = nm.b2 > 0 ? nm.r2 / nm.b2 : nm.r2;
    c->history.push_back(rel);
    prog.check(done, 0, rel);
    if (!std::isfinite(nm.r2) || !std::isfinite(nm.rinf)) {
      fill_info(info, GABP_ENUMERIC, done, lsw, 0, nm);
      return fail(GABP_ENUMERIC, "non-finite residual after sweep " + std::to_string(done));
    }
    if (rel <= tol) {
      fill_info(info, GABP_OK, done, lsw, 0, nm);
      return GABP_OK;
    }
  }
  fill_info(info, GABP_MAXSWEEPS, done, lsw, 0, nm);
  return GABP_MAXSWEEPS;
}

// FP32 mean messages inside FP64 iterative refinement.
//   x = 0, r = b; loop: stop at ||r||_2/||b||_2 <= tol; s = ||r||_inf; inner GaBP on
//   A d = r / s in FP32 from zero messages, checked every check_every sweeps through the
//   FP64 residual of x + s d; the inner solve ends when that residual fell by
//   ir_inner_tol, met tol, stopped improving, or hit the caps; then x += s d, r = that
//   residual.
int solve_ir(gabp_ctx* c, int T, const double* b, double* x, double tol, int max_sweeps,
             gabp_info* info, hipStream_t s) {
  int st;
  const bool had = c->pre[T].valid;
  if ((st = ensure_pre(c, T, s)) != GABP_OK) return st;
  const int lsw = had ? 0 : c->pre[T].sweeps;
  if ((st = ensure_msg32(c, s)) != GABP_OK) return st;
  const int64_t n = c->L.n;
  GABP_HIP(launch_fill64(x, n, 0.0, s));
  // three FP64 residual buffers: the accepted residual, the best trial, the next trial
  double* buf[3] = {c->r, c->r2, c->e};
  int ir = 0;
  // r = b - A 0 = b, with its norms
  if ((st = residual(c, T, b, x, nullptr, nullptr, buf[ir], s)) != GABP_OK) return st;
  Norms nm;
  if ((st = read_norms(c, s, &nm)) != GABP_OK) return st;
  if (!std::isfinite(nm.r2)) return fail(GABP_EINVAL, "non-finite right-hand side");
  const double bn = nm.b2;
  int total = 0, outer = 0;
  c->history.clear();
  Progress prog(c->opt.progress_s);
  double* scale = c->red + 4;   // device copy of s for this outer step
  while (true) {
    const double rel = bn > 0 ? nm.r2 / bn : nm.r2;
    if (rel <= tol || nm.r2 == 0.0) {
      fill_info(info, GABP_OK, total, lsw, outer, nm);
      return GABP_OK;
    }
    if (total >= max_sweeps) break;
    // s = ||r||_inf of the accepted residual (the device copy of max|r| belongs to the
    // last trial, which need not be the one kept); host_red[7] is read by no check
    c->host_red[7] = nm.rinf;
    GABP_HIP(hipMemcpyAsync(scale, c->host_red + 7, sizeof(double), hipMemcpyHostToDevice, s));
    GABP_HIP(launch_cast_scaled(c->r32, buf[ir], scale, n, s));
    if ((st = prep_rhs32(c, c->r32, s)) != GABP_OK) return st;
    if ((st = reset_messages32(c, s)) != GABP_OK) return st;
    const double rn = nm.r2;
    double best = rn;
    Norms nbest = nm;
    int ibest = -1, itry = (ir + 1) % 3;
    int inner = 0, since_best = 0;
    const bool rb = in_place(c);
    while (true) {
      const int k = std::min({c->opt.check_every, max_sweeps - total, c->opt.ir_max_inner - inner});
      if ((st = maybe_inject(c, total, true, s)) != GABP_OK) return st;
      const int start = c->parity32;
      const bool fresh = c->fresh32;
      double* rt = buf[itry];
      // one inner block: k FP32 sweeps, FP64 residual of x + s d, norms to the host
      st = run_block(c, *c->graphs, s, GraphKey{2, b, x, rt, start + 2 * fresh, k, T, 0.0},
                     [&](hipStream_t ss) -> int {
                       c->parity32 = start;
                       c->fresh32 = fresh;
                       int e = run_sweeps32(c, T, c->r32, k, c->d32, ss);
                       if (e != GABP_OK) return e;
                       e = residual(c, T, b, x, c->d32, scale, rt, ss);
                       if (e != GABP_OK) return e;
                       GABP_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double),
                                               hipMemcpyDeviceToHost, ss));
                       return GABP_OK;
                     });
      if (st != GABP_OK) return st;
      c->parity32 = rb ? start : start ^ (sweep_launches(c, k) & 1);
      c->fresh32 = false;
      inner += k;
      total += k;
      Norms nt;
      GABP_HIP(hipStreamSynchronize(s));
      host_norms(c, &nt);
      c->history.push_back(bn > 0 ? nt.r2 / bn : nt.r2);
      prog.check(total, outer, bn > 0 ? nt.r2 / bn : nt.r2);
      if (!std::isfinite(nt.r2)) {
        fill_info(info, GABP_ENUMERIC, total, lsw, outer, nt);
        return fail(GABP_ENUMERIC, "non-finite residual in iterative refinement");
      }
      // GaBP residuals are not monotone (a restart from zero messages first amplifies
      // rough residual components for a while): keep the best trial, and declare the FP32
      // floor only once the residual has improved and then shown no new best for
      // kPatience checks
      constexpr int kPatience = 8;
      if (nt.r2 < best) {
        best = nt.r2;
        nbest = nt;
        ibest = itry;
        itry = 3 - ir - ibest;
        GABP_HIP(hipMemcpyAsync(c->dbest32, c->d32, n * sizeof(float), hipMemcpyDeviceToDevice, s));
        since_best = 0;
      } else {
        ++since_best;
      }
      if (best <= c->opt.ir_inner_tol * rn || (bn > 0 ? best / bn : best) <= tol ||
          (ibest >= 0 && since_best >= kPatience) || inner >= c->opt.ir_max_inner ||
          total >= max_sweeps)
        break;
    }
    if (ibest < 0) {   // the FP32 inner solve could not reduce this residual at all
      fill_info(info, GABP_MAXSWEEPS, total, lsw, outer, nm);
      return fail(GABP_MAXSWEEPS, "iterative refinement stagnated");
    }
    GABP_HIP(launch_axpy32(x, c->dbest32, scale, n, s));   // x += s d_best
    ir = ibest;
    nm = nbest;
    ++outer;
  }
  fill_info(info, GABP_MAXSWEEPS, total, lsw, outer, nm);
  return GABP_MAXSWEEPS;
}

// The caller's b and x are staged through context-owned buffers, so the recorded check
// blocks (which bake in their buffer addresses) are reused across calls whatever tensors
// the caller passes.
int solve_any(gabp_ctx* c, int T, const double* b, double* x, double tol, int32_t max_sweeps,
              gabp_info* info, hipStream_t s) {
  if (!c || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  if (max_sweeps < 1 || !(tol >= 0.0)) return fail(GABP_EINVAL, "max_sweeps < 1 or tol < 0");
  if (seq_mode(c))
    return fail(GABP_ENOTSUPP, "solves need the precision messages of every sweep: use the "
                               "joint or the converged precomputed mode");
  GABP_HIP(hipSetDevice(c->device));
  const int64_t n = c->L.n;
  if (!c->bsol) {
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->bsol), n * sizeof(double)));
    GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->xsol), n * sizeof(double)));
  }
  GABP_HIP(hipMemcpyAsync(c->bsol, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  const int st = c->opt.precision == GABP_F32_IR
                     ? solve_ir(c, T, c->bsol, c->xsol, tol, max_sweeps, info, s)
                     : solve64(c, T, c->bsol, c->xsol, tol, max_sweeps, info, s);
  if (st == GABP_OK || st == GABP_MAXSWEEPS || st == GABP_ENUMERIC)
    GABP_HIP(hipMemcpyAsync(x, c->xsol, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return st;
}

}  // namespace

namespace gabp {
int precompute(gabp_ctx* c, int T, hipStream_t s) { return ensure_pre(c, T, s); }
}  // namespace gabp

extern "C" {

int gabp_solve(gabp_ctx* c, const double* b, double* x, double tol, int32_t max_sweeps,
               gabp_info* info, hipStream_t s) {
  return solve_any(c, 0, b, x, tol, max_sweeps, info, s);
}

int gabp_solve_transposed(gabp_ctx* c, const double* g, double* lam, double tol,
                          int32_t max_sweeps, gabp_info* info, hipStream_t s) {
  return solve_any(c, 1, g, lam, tol, max_sweeps, info, s);
}

int gabp_precompute_lambda(gabp_ctx* c, int32_t transposed, int32_t* sweeps_out,
                           hipStream_t s) {
  if (!c) return fail(GABP_EINVAL, "NULL context");
  const int T = transposed ? 1 : 0;
  c->pre[T].valid = false;
  int st = ensure_pre(c, T, s);
  if (st != GABP_OK) return st;
  GABP_HIP(hipStreamSynchronize(s));
  if (sweeps_out) *sweeps_out = c->pre[T].sweeps;
  return GABP_OK;
}

int gabp_sweeps(gabp_ctx* c, const double* b, double* x, int32_t sweeps, int32_t reset,
                int32_t transposed, hipStream_t s) {
  if (!c || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  if (sweeps < 1) return fail(GABP_EINVAL, "sweeps must be >= 1");
  const int T = transposed ? 1 : 0;
  int st;
  if (seq_mode(c) && T != 0)
    return fail(GABP_ENOTSUPP, "per-sweep precision messages are kept for A only");
  if (c->opt.precision == GABP_F32_IR) {
    // FP32 mean-only sweeps on fp32(b) with the FP32 copy of the precomputed Lt
    const bool fresh = !has_msg32(c);
    if (seq_mode(c)) {
      st = ensure_seq(c, (reset || fresh ? 0 : c->seq_pos32) + sweeps, s);
    } else {
      st = ensure_pre(c, T, s);
    }
    if (st != GABP_OK) return st;
    if ((st = ensure_msg32(c, s)) != GABP_OK) return st;
    GABP_HIP(launch_cast_scaled(c->r32, b, nullptr, c->L.n, s));
    if ((st = prep_rhs32(c, c->r32, s)) != GABP_OK) return st;
    if ((reset || fresh) && (st = reset_messages32(c, s)) != GABP_OK) return st;
    return run_sweeps32(c, T, c->r32, sweeps, nullptr, s, x, true);
  }
  if (c->opt.mode == GABP_MODE_PRECOMP && (st = ensure_pre(c, T, s)) != GABP_OK) return st;
  if (seq_mode(c) && (st = ensure_seq(c, (reset ? 0 : c->seq_pos64) + sweeps, s)) != GABP_OK)
    return st;
  if (reset && (st = reset_messages64(c, s)) != GABP_OK) return st;
  if ((st = prep_rhs64(c, b, s)) != GABP_OK) return st;
  return run_sweeps64(c, T, b, sweeps, x, s);
}

int gabp_smooth(gabp_ctx* c, const double* b, double* x, int32_t mu, hipStream_t s) {
  if (!c || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  if (mu < 1) return fail(GABP_EINVAL, "mu must be >= 1");
  return gabp::smooth_from(c, b, x, mu, false, false, s);
}

}  // extern "C"

namespace gabp {

// Algorithm 3 with the residual either computed here or already in c->r (r_ready: the
// caller has just formed b - A x for this x into c->r with the same residual kernel), or
// not needed (x_zero: x is zero on entry and is not read; the error equation's right-hand
// side is b itself). The correction is added to x by the last sweep itself (stored, for
// x_zero).
int smooth_from(gabp_ctx* c, const double* b, double* x, int mu, bool r_ready, bool x_zero,
                hipStream_t s) {
  int st;
  if (seq_mode(c) && (st = ensure_seq(c, mu, s)) != GABP_OK) return st;
  if (c->opt.precision == GABP_F32_IR) {
    if (!seq_mode(c) && (st = ensure_pre(c, 0, s)) != GABP_OK) return st;
    if ((st = ensure_msg32(c, s)) != GABP_OK) return st;
    if (x_zero) {
      GABP_HIP(launch_cast_scaled(c->r32, b, nullptr, c->L.n, s));
    } else if (r_ready) {
      GABP_HIP(launch_cast_scaled(c->r32, c->r, nullptr, c->L.n, s));
    } else if ((st = residual(c, 0, b, x, nullptr, nullptr, nullptr, s, false, c->r32)) !=
               GABP_OK) {
      return st;
    }
    if ((st = prep_rhs32(c, c->r32, s)) != GABP_OK) return st;
    if ((st = reset_messages32(c, s)) != GABP_OK) return st;
    return run_sweeps32(c, 0, c->r32, mu, nullptr, s, x, x_zero);
  }
  if (!x_zero && !r_ready &&
      (st = residual(c, 0, b, x, nullptr, nullptr, c->r, s, false)) != GABP_OK)
    return st;
  const double* rhs = x_zero ? b : c->r;
  if (c->opt.mode == GABP_MODE_PRECOMP && (st = ensure_pre(c, 0, s)) != GABP_OK) return st;
  if ((st = reset_messages64(c, s)) != GABP_OK) return st;
  if ((st = prep_rhs64(c, rhs, s)) != GABP_OK) return st;
  return run_sweeps64(c, 0, rhs, mu, nullptr, s, x, x_zero);
}

}  // namespace gabp

extern "C" {

int gabp_residual(gabp_ctx* c, const double* b, const double* x, double* r,
                  int32_t transposed, double* norms, hipStream_t s) {
  if (!c || !b || !x) return fail(GABP_EINVAL, "NULL argument");
  int st = residual(c, transposed ? 1 : 0, b, x, nullptr, nullptr, r, s);
  if (st != GABP_OK) return st;
  if (norms) {
    Norms nm;
    if ((st = read_norms(c, s, &nm)) != GABP_OK) return st;
    norms[0] = nm.r2;
    norms[1] = nm.rinf;
    norms[2] = nm.b2;
  }
  return GABP_OK;
}

int gabp_adjoint_scatter(gabp_ctx* c, const double* lam, const double* x, double* G,
                         int32_t nparam, const int32_t* jptr, const int32_t* jnnz,
                         const double* jw, double* dtheta, hipStream_t s) {
  if (!c || !lam || !x) return fail(GABP_EINVAL, "NULL argument");
  if (jptr && (!jnnz || !jw || !dtheta || nparam < 0))
    return fail(GABP_EINVAL, "incomplete parameter Jacobian");
  if (G) GABP_HIP(launch_entry_grad(&c->L, lam, x, G, s));
  if (jptr)
    GABP_HIP(launch_param_reduce(nparam, jptr, jnnz, jw, lam, x, c->L.csr_row, c->L.csr_col,
                                 dtheta, s));
  return GABP_OK;
}

// ---- checkpoints ----------------------------------------------------------------------
namespace {
// The header names what the message positions depend on (layout, schedule, mode,
// precision), so a blob only loads into a context that lays its messages out the same way.
struct StateHeader {
  uint64_t magic;
  int64_t n, epad;
  int32_t pre_valid[2], pre_sweeps[2];
  int32_t has32, pad;
  uint64_t layout_hash;
  int32_t schedule, mode, precision, seq_pos64, seq_pos32, pad2;
};
constexpr uint64_t kMagic = 0x6761627073743032ull;      // "gabpst02"
constexpr uint64_t kLineMagic = 0x676162706c6e3032ull;  // "gabpln02"

StateHeader make_header(const gabp_ctx* c, uint64_t magic, bool pre0, bool pre1, bool has32) {
  StateHeader h{};
  h.magic = magic;
  h.n = c->L.n;
  h.epad = c->L.epad;
  h.pre_valid[0] = pre0;
  h.pre_valid[1] = pre1;
  h.pre_sweeps[0] = c->pre[0].sweeps;
  h.pre_sweeps[1] = c->pre[1].sweeps;
  h.has32 = has32;
  h.layout_hash = c->L.hash;
  h.schedule = c->opt.schedule;
  h.mode = c->opt.mode;
  h.precision = c->opt.precision;
  h.seq_pos64 = c->seq_pos64;
  h.seq_pos32 = c->seq_pos32;
  return h;
}

// Line schedules: the header, then the arrays listed by line_state_arrays.
int line_get_state(gabp_ctx* c, void* dst, size_t* bytes, hipStream_t s) {
  const bool pre[2] = {c->pre[0].valid, c->pre[1].valid};
  const bool has32 = line_has32(c);
  std::vector<StateArray> arr;
  int st;
  if (dst && ((st = line_zero_incoming64(c, s)) != GABP_OK ||
              (st = line_zero_incoming32(c, s)) != GABP_OK))
    return st;
  if ((st = line_state_arrays(c, has32, pre, false, &arr)) != GABP_OK) return st;
  size_t need = sizeof(StateHeader);
  for (const auto& a : arr) need += a.bytes;
  if (!dst) {
    *bytes = need;
    return GABP_OK;
  }
  if (*bytes < need) return fail(GABP_EINVAL, "state buffer too small");
  const StateHeader h = make_header(c, kLineMagic, pre[0], pre[1], has32);
  char* p = static_cast<char*>(dst);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  for (const auto& a : arr) {
    GABP_HIP(hipMemcpyAsync(p, a.p, a.bytes, hipMemcpyDeviceToHost, s));
    p += a.bytes;
  }
  GABP_HIP(hipStreamSynchronize(s));
  *bytes = need;
  return GABP_OK;
}

int line_set_state(gabp_ctx* c, const StateHeader& h, const char* p, size_t bytes,
                   hipStream_t s) {
  const bool pre[2] = {h.pre_valid[0] != 0, h.pre_valid[1] != 0};
  std::vector<StateArray> arr;
  int st;
  if ((st = line_state_arrays(c, h.has32 != 0, pre, true, &arr)) != GABP_OK) return st;
  size_t need = sizeof(StateHeader);
  for (const auto& a : arr) need += a.bytes;
  if (bytes < need) return fail(GABP_EINVAL, "state blob truncated");
  for (const auto& a : arr) {
    GABP_HIP(hipMemcpyAsync(a.p, p, a.bytes, hipMemcpyHostToDevice, s));
    p += a.bytes;
  }
  for (int T = 0; T < 2; ++T) {
    c->pre[T].valid = pre[T];
    c->pre[T].sweeps = pre[T] ? h.pre_sweeps[T] : 0;
  }
  c->fresh64 = false;
  c->fresh32 = false;
  GABP_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}
}  // namespace

int gabp_get_state(gabp_ctx* c, void* dst, size_t* bytes, hipStream_t s) {
  if (!c || !bytes) return fail(GABP_EINVAL, "NULL argument");
  if (c->lines) return line_get_state(c, dst, bytes, s);
  const Layout& L = c->L;
  const size_t E = static_cast<size_t>(L.epad + 1), N = static_cast<size_t>(L.n);
  size_t need = sizeof(StateHeader) + 2 * E * sizeof(double);
  for (int T = 0; T < 2; ++T)
    if (c->pre[T].valid) need += E * (sizeof(double) + sizeof(float)) + N * (sizeof(double) + sizeof(float));
  if (c->msg32[0]) need += E * sizeof(float);
  if (!dst) {
    *bytes = need;
    return GABP_OK;
  }
  if (*bytes < need) return fail(GABP_EINVAL, "state buffer too small");
  const StateHeader h = make_header(c, kMagic, c->pre[0].valid, c->pre[1].valid,
                                    c->msg32[0] != nullptr);
  char* p = static_cast<char*>(dst);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  auto get = [&](const void* src, size_t nb) -> int {
    GABP_HIP(hipMemcpyAsync(p, src, nb, hipMemcpyDeviceToHost, s));
    p += nb;
    return GABP_OK;
  };
  auto zeros = [&](size_t nb) {   // a reset state: the buffers are logically zero
    std::memset(p, 0, nb);
    p += nb;
  };
  int st;
  if (c->fresh64) {
    zeros(2 * E * sizeof(double));
  } else if ((st = get(c->lam[c->parity], E * sizeof(double))) ||
             (st = get(c->msg[c->parity], E * sizeof(double)))) {
    return st;
  }
  for (int T = 0; T < 2; ++T)
    if (c->pre[T].valid) {
      if ((st = get(c->pre[T].lamout, E * sizeof(double))) || (st = get(c->pre[T].S, N * sizeof(double))) ||
          (st = get(c->pre[T].lamout32, E * sizeof(float))) || (st = get(c->pre[T].invS32, N * sizeof(float))))
        return st;
    }
  if (c->msg32[0]) {
    if (c->fresh32) zeros(E * sizeof(float));
    else if ((st = get(c->msg32[c->parity32], E * sizeof(float)))) return st;
  }
  GABP_HIP(hipStreamSynchronize(s));
  *bytes = need;
  return GABP_OK;
}

int gabp_set_state(gabp_ctx* c, const void* src, size_t bytes, hipStream_t s) {
  if (!c || !src || bytes < sizeof(StateHeader)) return fail(GABP_EINVAL, "bad state");
  StateHeader h;
  std::memcpy(&h, src, sizeof(h));
  const Layout& L = c->L;
  if (h.magic != (c->lines ? kLineMagic : kMagic) || h.n != L.n || h.epad != L.epad ||
      h.layout_hash != L.hash || h.schedule != c->opt.schedule || h.mode != c->opt.mode ||
      h.precision != c->opt.precision)
    return fail(GABP_EINVAL, "state was taken from a different layout, schedule or mode");
  c->seq_pos64 = h.seq_pos64;
  c->seq_pos32 = h.seq_pos32;
  if (c->lines)
    return line_set_state(c, h, static_cast<const char*>(src) + sizeof(h), bytes, s);
  const size_t E = static_cast<size_t>(L.epad + 1), N = static_cast<size_t>(L.n);
  size_t need = sizeof(StateHeader) + 2 * E * sizeof(double);
  for (int T = 0; T < 2; ++T)
    if (h.pre_valid[T]) need += E * (sizeof(double) + sizeof(float)) + N * (sizeof(double) + sizeof(float));
  if (h.has32) need += E * sizeof(float);
  if (bytes < need) return fail(GABP_EINVAL, "state blob truncated");
  const char* p = static_cast<const char*>(src) + sizeof(h);
  auto put = [&](void* d, size_t nb) -> int {
    GABP_HIP(hipMemcpyAsync(d, p, nb, hipMemcpyHostToDevice, s));
    p += nb;
    return GABP_OK;
  };
  int st;
  c->parity = 0;
  c->fresh64 = false;
  if ((st = put(c->lam[0], E * sizeof(double))) || (st = put(c->msg[0], E * sizeof(double)))) return st;
  for (int T = 0; T < 2; ++T) {
    if (!h.pre_valid[T]) {
      c->pre[T].valid = false;
      continue;
    }
    Precomp& P = c->pre[T];
    if (!P.lamout) {
      GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.lamout), E * sizeof(double)));
      GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.S), N * sizeof(double)));
      GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.lamout32), E * sizeof(float)));
      GABP_HIP(hipMalloc(reinterpret_cast<void**>(&P.invS32), N * sizeof(float)));
    }
    if ((st = put(P.lamout, E * sizeof(double))) || (st = put(P.S, N * sizeof(double))) ||
        (st = put(P.lamout32, E * sizeof(float))) || (st = put(P.invS32, N * sizeof(float))))
      return st;
    P.valid = true;
    P.sweeps = h.pre_sweeps[T];
  }
  if (h.has32) {
    if ((st = ensure_msg32(c, s)) != GABP_OK) return st;
    c->parity32 = 0;
    c->fresh32 = false;
    if ((st = put(c->msg32[0], E * sizeof(float)))) return st;
  }
  GABP_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_get_messages(gabp_ctx* c, double* lam, double* msg, hipStream_t s) {
  if (!c) return fail(GABP_EINVAL, "NULL context");
  if (c->lines) return fail(GABP_ENOTSUPP, "line schedules keep line messages, not edge messages");
  if (c->batch) return fail(GABP_ENOTSUPP, "batched contexts keep one message set per rhs");
  const double* L = nullptr;
  bool outgoing = false;
  const bool f32 = c->opt.precision == GABP_F32_IR;
  if (c->opt.mode == GABP_MODE_JOINT && !f32) {
    if (!c->fresh64) L = c->lam[c->parity];
  } else if (seq_mode(c)) {
    const int k = f32 ? c->seq_pos32 : c->seq_pos64;   // the Lt of sweep k is in use
    if (k > 0) {
      if (!c->seq.valid || k > c->seq.depth)
        return fail(GABP_EINVAL, "per-sweep precision messages not computed");
      L = c->seq.lamout[k - 1];
      outgoing = true;
    }
  } else {
    if (!c->pre[0].valid) return fail(GABP_EINVAL, "precision messages not computed yet");
    L = c->pre[0].lamout;
    outgoing = true;
  }
  const double* M = nullptr;
  const float* M32 = nullptr;
  if (f32) {
    if (c->msg32[0] && !c->fresh32) M32 = c->msg32[c->parity32];
  } else if (!c->fresh64) {
    M = c->msg[c->parity];
  }
  GABP_HIP(launch_gather_messages(&c->L, L, outgoing, M, M32, lam, msg, s));
  return GABP_OK;
}

int gabp_residual_history(const gabp_ctx* c, double* out, int32_t cap, int32_t* count) {
  if (!c || !count) return fail(GABP_EINVAL, "NULL argument");
  if (cap < 0) return fail(GABP_EINVAL, "cap < 0");
  const int32_t m = static_cast<int32_t>(c->history.size());
  *count = m;
  if (out)
    for (int32_t i = 0; i < std::min(m, cap); ++i) out[i] = c->history[i];
  return GABP_OK;
}

int gabp_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  if (!src || !dst || bytes < 0 || bytes % 16 != 0)
    return fail(GABP_EINVAL, "copy probe needs non-NULL pointers and a multiple of 16 bytes");
  GABP_HIP(launch_copy_probe(src, dst, bytes, s));
  return GABP_OK;
}

}  // extern "C"
