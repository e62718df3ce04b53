// Line GaBP: the two-layer region iteration (Sec. 3, Algorithm 2) whose large regions are
// the rows and the columns of a 2-D grid and whose small regions are the single nodes
// (Fig. two_layers_network). Every node receives one message from its row and one from
// its column; a line's update is a tridiagonal elimination from both ends:
//
//   d_t = A_tt + Lambda_in(t),  c_t = b_t + m_in(t)      (the other line's messages)
//   f_0 = d_0, g_0 = c_0;   f_t = d_t - lo_t hi_{t-1} / f_{t-1},  g_t = c_t - lo_t g_{t-1} / f_{t-1}
//   h_L = d_L, q_L = c_L;   h_t = d_t - hi_t lo_{t+1} / h_{t+1},  q_t = c_t - hi_t q_{t+1} / h_{t+1}
//   Lambda_out(t) = (f_t - d_t) + (h_t - d_t),   m_out(t) = (g_t - c_t) + (q_t - c_t)
//
// (lo_t / hi_t: coupling of position t to its predecessor / successor along the line).
// The read-off is Algorithm 2's [x]_L of the last line updated that contains the node, its
// column: x = (c_t + m_out(t)) / (d_t + Lambda_out(t)) of the column update, formed in the
// column layout right after that update and transposed into the row layout.
// f_t + h_t - d_t is 1 / (T^{-1})_tt of the line's tridiagonal matrix T and g_t + q_t - c_t
// is that Schur complement times x_t, so these are eq. Two_layers_GaBP_rules with the
// line's own diagonal and incoming messages removed. With frozen precision messages the
// pivots are constants and the mean recurrences are linear: g_t = c_t - alpha_t g_{t-1},
// q_t = c_t - beta_t q_{t+1}, alpha_t = lo_t / f_{t-1}, beta_t = hi_t / h_{t+1}.
//
// GPU form: one 256-thread block per line, each thread owns NPL consecutive positions in
// registers. The forward and backward recurrences are first-order in projective form
// (theta_t = d_t theta_{t-1} - p_t theta_{t-2}, G_t = c_t theta_{t-1} - lo_t G_{t-1},
// f_t = theta_t / theta_{t-1}, g_t = G_t / theta_{t-1}), i.e. products of 3x3 matrices, so
// a block-wide scan of the per-thread products gives every thread its incoming state;
// each thread then runs the plain ratio recurrences over its own positions. Lines are
// stored line-major (row layout: index y*nx + x for the rows; column layout: x*ny + y for
// the columns), so every line is contiguous; the messages a line sends are transposed
// into the other layout by a tiled LDS transpose after each update.
#pragma once

#include <vector>

#include "gabp_internal.h"

namespace gabp {

constexpr int kLineThreads = 256;
constexpr int kLineMaxLen = 16 * kLineThreads;   // NPL <= 16 positions per thread

// One orientation: `nlines` lines of `len` positions, line-major.
struct LineSide {
  int nlines = 0, len = 0;
  double* diag = nullptr;                  // [n] A_tt
  double* lo[2] = {nullptr, nullptr};      // [T][n] coupling to the predecessor (A, A^T)
  double* hi[2] = {nullptr, nullptr};      // [T][n] coupling to the successor
  int32_t* diag_src = nullptr;             // [n] CSR index of each value (-1: none)
  int32_t* lo_src[2] = {nullptr, nullptr};
  int32_t* hi_src[2] = {nullptr, nullptr};
  // joint FP64 messages sent by this orientation's lines: in this layout (written by the
  // line update) and transposed into the other layout (read by the other orientation)
  double* lam_own = nullptr;
  double* m_own = nullptr;
  double* lam_x = nullptr;
  double* m_x = nullptr;
  // frozen precision messages: recurrence multipliers per transposition
  double* alpha[2] = {nullptr, nullptr};
  double* beta[2] = {nullptr, nullptr};
  float* alpha32[2] = {nullptr, nullptr};
  float* beta32[2] = {nullptr, nullptr};
  // FP32 mean messages (refinement inner sweeps)
  float* m32_own = nullptr;
  float* m32_x = nullptr;
};

struct LineLayout {
  int nx = 0, ny = 0;
  int64_t n = 0;
  bool alt = false;                        // rows first, then columns from the new messages
  LineSide side[2];                        // 0: rows (row layout), 1: columns (column layout)
  double* bcol = nullptr;                  // [n] right-hand side in the column layout
  float* bcol32 = nullptr;
  double* zero = nullptr;                  // [n] zeros (right-hand side of the Lt phase)
  double* invS[2] = {nullptr, nullptr};    // [T][n] 1 / (T^{-1})_tt of the frozen column
  float* invS32[2] = {nullptr, nullptr};   //   systems, column layout (frozen read-off)
  double* xcol = nullptr;                  // [n] read-off in the column layout
  float* xcol32 = nullptr;
  double* partials = nullptr;              // [2 * (nx + ny)] per-line max|dLambda|, max|Lambda|
  // mean-only line sweeps with non-temporal loads: FP64 / FP32 sweep bytes (40 / 20 B per
  // node and orientation) above the last-level cache
  bool nt64 = false, nt32 = false;
};

// Arguments of one orientation's line update.
struct LineArgs {
  int nlines, len;
  const double* diag;
  const double* lo;
  const double* hi;
  const double* b;        // right-hand side in this layout
  const double* lam_in;   // the other orientation's messages, this layout
  const double* m_in;
  double* lam_out;        // null: messages not written (pivots only)
  double* m_out;
  double* alpha;          // non-null: write alpha_t, beta_t (frozen-Lambda multipliers)
  double* beta;
  float* alpha32;
  float* beta32;
  double* invS;           // with alpha: also 1 / (T^{-1})_tt = 1 / (f_t + h_t - d_t), if non-null
  float* invS32;
  double* partials;       // non-null: per line max|Lambda_out - old|, max|Lambda_out|
};

template <typename T>
struct LineMeanArgs {
  int nlines, len;
  const T* alpha;
  const T* beta;
  const T* b;
  const T* m_in;
  T* m_out;
  bool nt = false;   // non-temporal loads of the streamed arrays (the sweep exceeds the LLC)
};

template <typename T>
struct TransposeJob {
  const T* src;   // rows x cols, row-major
  T* dst;         // cols x rows, row-major
  int rows, cols;
};

// kernels_line.hip
hipError_t launch_line_joint(const LineArgs* sides, int nsides, hipStream_t s);
hipError_t launch_line_mean64(const LineMeanArgs<double>* sides, int nsides, hipStream_t s);
hipError_t launch_line_mean32(const LineMeanArgs<float>* sides, int nsides, hipStream_t s);
hipError_t launch_transpose64(const TransposeJob<double>* jobs, int njobs, hipStream_t s);
hipError_t launch_transpose32(const TransposeJob<float>* jobs, int njobs, hipStream_t s);
hipError_t launch_line_readoff64(int64_t n, const double* b, const double* diag,
                                 const double* lam_r, const double* m_r, const double* lam_c,
                                 const double* m_c, const double* invS, double* x,
                                 hipStream_t s);
hipError_t launch_line_readoff32(int64_t n, const float* b, const float* m_r, const float* m_c,
                                 const float* invS, float* x, hipStream_t s);
hipError_t launch_gather_values(int64_t n, const int32_t* src, const double* val, double* dst,
                                hipStream_t s);

// line.cpp
int line_setup(gabp_ctx* c, int nx, int ny, const int32_t* rowptr, const int32_t* col,
               const double* val);
void line_destroy(LineLayout* L);
int line_update_values(gabp_ctx* c, const double* val, hipStream_t s);
int line_reset64(gabp_ctx* c, hipStream_t s);
int line_ensure32(gabp_ctx* c, hipStream_t s);   // FP32 message buffers (zeroed)
bool line_has32(const gabp_ctx* c);
int line_reset32(gabp_ctx* c, hipStream_t s);
// write out the zeros a reset only marked (no-op unless c->fresh64 / c->fresh32)
int line_zero_incoming64(gabp_ctx* c, hipStream_t s);
int line_zero_incoming32(gabp_ctx* c, hipStream_t s);
int line_rhs64(gabp_ctx* c, const double* b, hipStream_t s);
int line_rhs32(gabp_ctx* c, const float* b, hipStream_t s);
int line_sweep64(gabp_ctx* c, int T, const double* b, double* x, hipStream_t s);
int line_sweep32(gabp_ctx* c, int T, const float* b, float* x, hipStream_t s);
int line_precompute(gabp_ctx* c, int T, hipStream_t s);

// Checkpoint: the device arrays of the iteration state in a fixed order -- the joint FP64
// messages of both orientations (own layout and the other layout's copy), the FP32 mean
// messages if has32, and per transposition T with pre[T] the frozen multipliers (FP64 and
// FP32) and read-off factors. alloc: allocate what a restore needs and is missing.
struct StateArray {
  void* p;
  size_t bytes;
};
int line_state_arrays(gabp_ctx* c, bool has32, const bool pre[2], bool alloc,
                      std::vector<StateArray>* out);

}  // namespace gabp
