// Internal declarations shared by the host drivers and the HIP kernels of libgabp.
//
// Layout ("SELL-64 over the symmetrised pattern"):
//  * Every row j owns one slot per neighbour i of the symmetrised off-diagonal pattern
//    {i != j : A_ji != 0 or A_ij != 0}, columns ascending. Slot (j,i) holds the message
//    i -> j that row j *receives* (Lt_ij, m_ij), plus val = A_ji (row j's own coefficient,
//    used by r = b - A x) and aT = A_ij (the coefficient of the message j -> i that row j
//    *sends*, and of Lt_ij in Sigma_j). A missing entry is stored as 0, which makes the
//    corresponding message exactly zero (Sec. 2.3: if A_jk = 0, x_k is not eliminated).
//  * Rows are grouped into slices of 64 lanes (one wavefront); slice s occupies
//    [sptr[s], sptr[s+1]) and stores slot k of the row at lane 64 s + l at
//    sptr[s] + 64 k + l, so the 64 lanes of a wavefront touch 64 consecutive elements for
//    every k. Lane t holds row t, or with a colouring the colour-major order of Layout.
//  * rev[p] is the position of the reverse slot (i,j); padding slots are their own
//    reverse (a zero message is written there every sweep). Position epad (one past the
//    padded slots) is allocated but holds no message.
//  * The sweep is written "push" style, as Algorithm 1 is: the thread of row j reads its
//    own incoming messages (contiguous), forms Sigma_j and M_j, reads off x_j and writes
//    every outgoing message j -> i straight into the receiver's slot rev[p].
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/gabp.h"

namespace gabp {

struct Batch;
struct GraphCache;
struct LineLayout;
constexpr int kSlice = 64;      // rows per slice = wavefront size on CDNA
constexpr int kBlock = 256;     // threads per block for row kernels (4 slices)
constexpr int kRedBlock = 256;      // threads per block for reductions
constexpr int kRevSelf16 = -32768;  // classed rev16: the slot is its own reverse
constexpr int kMaxColours = 8;  // colour classes of the coloured schedule
// Layout::row_slot packs a row's first slot (below 2^29) and its slice width (below 8)
constexpr int kRowSlotShift = 29;
constexpr unsigned kRowSlotMask = (1u << kRowSlotShift) - 1u;
constexpr int kXcds = 8;   // XCDs of an MI355X (8 x 32 compute units, one L2 each)

// Tiles of the two-sweep (temporally blocked) flood kernels: Layout::tile_slices slices of
// 64 lanes per tile (a multiple of kTileUnit), handled by kTileOwnThreads threads (one lane
// per thread and kTileUnit slices, i.e. one or two lanes per thread) plus kHaloThreads
// threads for the tile's halo rows (a 5-point tile of 13 x 64 nodes has 154, of 26 x 64
// nodes 180), in one workgroup of kTileThreads; rows of at most kTileMaxWidth slots, so a
// tile's incoming messages fit in LDS (FP64 joint, 13 slices: 2 x 8 B x 13 x 64 x 4 =
// 52 KiB; FP64 mean-only, 13 slices: 26 KiB; FP32 mean-only, 26 slices: 26 KiB)
constexpr int kTileUnit = 13;
constexpr int kTileOwnThreads = kTileUnit * kSlice;
constexpr int kHaloThreads = 192;
constexpr int kTileThreads = kTileOwnThreads + kHaloThreads;
constexpr int kTileMaxWidth = 4;

struct Precomp {
  bool valid = false;
  int sweeps = 0;
  double* lamout = nullptr;    // [epad] Lt*_ji of the message j -> i, stored at slot (j,i)
  double* S = nullptr;         // [n] Sigma*_j
  float* lamout32 = nullptr;   // [epad] FP32 copy of lamout
  float* invS32 = nullptr;     // [n] FP32 of 1/Sigma* (computed in FP64, rounded once)
};

// Precision messages of the first sweeps after a message reset (mode GABP_MODE_PRECOMP_SEQ).
// They do not depend on the right-hand side, so a smoother that restarts from zero messages
// needs exactly these at every call; entry s - 1 holds what sweep s uses.
struct SeqPrecomp {
  bool valid = false;            // the stored entries belong to the current values of A
  int depth = 0;                 // entries computed
  std::vector<double*> lamout;   // [epad + 1] Lt sent in sweep s, at the sender's slot (j,i)
  std::vector<double*> S;        // [n] Sigma_j of sweep s's read-off
  std::vector<float*> lamout32;  // FP32 copies (rounded once from FP64)
  std::vector<float*> invS32;    // FP32 of 1 / Sigma_j (computed in FP64)
};

struct Layout {
  int32_t n = 0;
  int64_t nnz = 0;
  int64_t slots = 0;      // directed message slots (symmetrised pattern)
  int64_t epad = 0;       // padded slot count
  int32_t nslices = 0;
  int32_t max_width = 0;  // max slots per row
  // non-temporal hints on the per-slot streams of the FP64 / FP32 sweeps: they pay off
  // once a sweep's footprint exceeds the last-level cache and cost time below it
  bool stream_hints = false;
  bool stream_hints32 = false;
  // tiled kernels only: non-temporal stores while the loads stay plain (a tile's halo reads
  // lines its neighbours load, and plain loads keep them in L2)
  bool store_hints = false;
  bool store_hints32 = false;
  // the residual kernel's streamed inputs (row slots, b, diag, columns, coefficients) with
  // non-temporal loads (x, which it gathers, stays plain): its bytes exceed the LLC
  bool res_hints = false;
  // threads per workgroup of the single-system sweep kernels: 64, 128 or 256 (1, 2 or 4
  // slices), picked by the autotuner
  int32_t block = kBlock;
  // device
  int32_t* sptr = nullptr;   // [nslices+1]
  int32_t* rev = nullptr;    // [epad]
  // rev16 in a two-class colour-major layout (rev16_classed): rev[p] - p - (first slot of
  // the other class - first slot of p's class), or kRevSelf16 for a padding slot (its own
  // reverse); a flood launch over such a layout reads rev instead
  bool rev16_classed = false;
  int16_t* rev16 = nullptr;  // [epad] rev[p] - p when every slot's reverse lies within
                             // int16 range (grid matrices); padding slots hold 0 (self)
  int32_t* col = nullptr;    // [epad]
  double* val = nullptr;     // [epad] A_ji at slot (j,i)
  double* aT = nullptr;      // [epad] A_ij at slot (j,i)
  double* diag = nullptr;    // [n]
  int32_t* val_src = nullptr;   // [epad] CSR index feeding val (-1: zero)
  int32_t* aT_src = nullptr;    // [epad] CSR index feeding aT (-1: zero)
  int32_t* diag_src = nullptr;  // [n]
  int32_t* csr_row = nullptr;   // [nnz] row of each stored entry (adjoint scatter)
  int32_t* csr_col = nullptr;   // [nnz]
  int32_t ncolours = 0;         // colour classes (1 + the largest colour), 0 without colours
  // Lanes: thread t of a row kernel serves lane t & 63 of slice t >> 6. Without colours lane
  // t holds row t (nlanes = n). With a colouring the lanes are colour-major: the rows of
  // colour 0 in ascending order, padded to whole slices, then those of colour 1, ..., so a
  // colour pass is one launch over the full slices of lanes [cstart[c], cstart[c+1]).
  // perm[t] = row held by lane t, -1 for a padding lane (null: identity).
  int32_t nlanes = 0;
  std::vector<int32_t> cstart;        // [ncolours + 1] first lane of each colour (host)
  std::vector<int32_t> cslot;         // [ncolours + 1] first slot of each colour (host)
  int32_t* perm = nullptr;            // [nlanes] or null
  int32_t* lane_of_row_d = nullptr;   // [n] lane of each row, the inverse of perm, or null
  std::vector<int32_t> lane_of_row;   // host copy of the inverse (empty: identity)
  // [n] for row-order kernels (the residual): first slot of row j | slice width << 29, or
  // null when a slot index or width does not fit
  int32_t* row_slot = nullptr;
  uint64_t hash = 0;                  // of the slot and lane layout (checkpoint check)
  // tiled layout (opt.tiles): lanes tile-major, tile t = lanes [t, t + 1) * tile_slices * 64;
  // halo of tile t = entries tile_halo[t * kHaloThreads ...] (the rows outside the tile that
  // send into it, {first slot, slots, row, 0}; entries past the halo have no slots)
  int32_t ntiles = 0;
  int32_t tile_slices = 0;            // 13 (FP64 sweeps) or 26 (FP32 mean-only sweeps)
  int32_t tile_slots_max = 0;         // largest slot range of one tile
  int4* tile_halo = nullptr;          // [ntiles * kHaloThreads]
  int32_t tiles_x = 0;                // tile columns (tile t sits at column t % tiles_x)
  int32_t grid_nx = 0, grid_ny = 0;   // the grid: node (x, y) is row y * grid_nx + x
  int32_t tile_strip = 1;             // tile columns per strip of the XCD-aware tile order
};

}  // namespace gabp

struct gabp_ctx {
  int device = 0;
  gabp_options opt{};
  gabp::Layout L;
  // message state: lam[parity], msg[parity] hold the current incoming messages
  double* lam[2] = {nullptr, nullptr};
  double* msg[2] = {nullptr, nullptr};
  float* msg32[2] = {nullptr, nullptr};
  int parity = 0;
  int parity32 = 0;
  gabp::Precomp pre[2];       // [0] A, [1] A^T
  gabp::SeqPrecomp seq;       // per-sweep Lt of A (mode GABP_MODE_PRECOMP_SEQ)
  int seq_pos64 = 0;          // sweeps since the last message reset, FP64 / FP32 messages
  int seq_pos32 = 0;
  // work vectors
  double* r = nullptr;        // [n]
  double* r2 = nullptr;       // [n]
  double* e = nullptr;        // [n]
  double* bsol = nullptr;     // [n] staged right-hand side of gabp_solve*
  double* xsol = nullptr;     // [n] staged iterate of gabp_solve*
  float* r32 = nullptr;       // [n]
  float* d32 = nullptr;       // [n]
  float* dbest32 = nullptr;   // [n] best inner correction of the current refinement step
  // reductions
  int32_t nred = 0;           // blocks of the residual kernel
  // per-block partials, shared by the residual kernel (3 per block of kRedBlock rows) and
  // the Lt-phase kernel (2 per block of kBlock lanes): [npartials], enough for both
  double* partials = nullptr;
  int64_t npartials = 0;
  double* red = nullptr;      // [8] device scalars: 0 ||r||2^2, 1 max|r|, 2 ||b||2^2,
                              // 3 max|r| again, 4 refinement scale, 5 max|dLt|, 6 max|Lt|
  unsigned long long* lmax = nullptr;  // [2] max|dLt|, max|Lt| as ordered bit patterns
  double* host_red = nullptr;          // pinned [8]
  gabp::Batch* batch = nullptr;        // set for contexts made by gabp_setup_batched
  gabp::GraphCache* graphs = nullptr;  // recorded check blocks
  gabp::LineLayout* lines = nullptr;   // set for the line schedules
  // fault injection (environment GABP_FAULT_INJECT=nan@sweep:k, read at set-up): before the
  // first check block that starts at or after sweep k, the incoming mean messages are
  // overwritten with NaN; -1 when off or already done
  // message buffers that are logically zero (reset) but not cleared: the next sweep of
  // that precision treats them as zero and writes every slot
  bool fresh64 = false;
  bool fresh32 = false;
  int32_t inject_nan_at = -1;
  // GABP_FAULT_INJECT=poison-outputs: every ping-pong sweep first fills its output message
  // buffers with NaN, so a slot the sweep does not write shows up in the next read-off
  bool poison_outputs = false;
  std::vector<double> history;         // ||r||_2 / ||b||_2 at every check of the last solve
};

namespace gabp {

// ---- error reporting ----
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
// CSR check of gabp_validate_csr (host only, validate.cpp)
int validate(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
             const double* val, const int32_t* rev);
// Algorithm 3 (gabp_smooth); r_ready: c->r already holds b - A x for this x; x_zero: x is
// zero on entry and not read (solve.cpp)
int smooth_from(gabp_ctx* c, const double* b, double* x, int mu, bool r_ready, bool x_zero,
                hipStream_t s);
#define GABP_HIP(call)                                           \
  do {                                                           \
    hipError_t _e = (call);                                      \
    if (_e != hipSuccess) return ::gabp::hip_fail(_e, #call);    \
  } while (0)

// Lt phase of the context (T = 1: for A^T), computed once and cached (solve.cpp)
int precompute(gabp_ctx* c, int T, hipStream_t s);
// device address of the allocation-free entry point's static array on device `dev`, which
// must be current; looked up once per device (noalloc.hip). out may be NULL.
int scratch_on(int dev, double** out);
// per-sweep Lt of the first `depth` sweeps after a reset (mode PRECOMP_SEQ, solve.cpp)
int ensure_seq(gabp_ctx* c, int depth, hipStream_t s);
void free_seq(gabp_ctx* c);

// ---- kernel launchers (kernels.hip) ----
struct SweepArgs {
  const Layout* L;
  const double* coef;       // aT (forward) or val (transposed)
  const double* b;
  const double* lam_in;
  const double* msg_in;
  double* lam_out;
  double* msg_out;
  double* x;                // null: no read-off written
  int colour;               // -1 all lanes, else only the lanes of that colour (in place)
  // >= 0: first sweep after a message reset; incoming slot p counts only if rev(p) < fresh
  // (the slots of the colours already updated in this sweep), else its message is zero
  int fresh = -1;
  double* xadd = nullptr;   // non-null: the read-off is added to xadd instead (x unused)
  bool xset = false;        // with xadd: stored into xadd instead of added
};
hipError_t launch_joint_sweep(const SweepArgs& a, hipStream_t s);

struct MeanArgs64 {
  const Layout* L;
  const double* lamout;
  const double* S;
  const double* b;
  const double* msg_in;
  double* msg_out;
  double* x;
  int colour;
  int fresh = -1;
  double* xadd = nullptr;   // non-null: the read-off is added to xadd instead (x unused)
  bool xset = false;        // with xadd: stored into xadd instead of added
};
hipError_t launch_mean_sweep64(const MeanArgs64& a, hipStream_t s);

struct MeanArgs32 {
  const Layout* L;
  const float* lamout;
  const float* invS;
  const float* b;
  const float* msg_in;
  float* msg_out;
  float* x;
  int colour;
  int fresh = -1;
  double* xadd = nullptr;   // non-null: the FP32 read-off, widened, is added to xadd
  bool xset = false;        // with xadd: stored into xadd instead of added
};
hipError_t launch_mean_sweep32(const MeanArgs32& a, hipStream_t s);

// Two flood sweeps in one launch on a tiled layout (L.ntiles > 0): joint (SweepArgs with
// colour -1) or mean-only with the Lt of the first sweep (lamA) and of the second (lamB,
// with SxB its Sigma or 1/Sigma); read-off (x, xadd) of the second sweep.
hipError_t launch_joint_pair(const SweepArgs& a, hipStream_t s);
template <typename T>
struct MeanPairArgs {
  const Layout* L;
  const T* lamA;
  const T* lamB;
  const T* SxB;
  const T* b;
  const T* msg_in;
  T* msg_out;
  T* x;
  int fresh = -1;
  double* xadd = nullptr;
  bool xset = false;
};
hipError_t launch_mean_pair64(const MeanPairArgs<double>& a, hipStream_t s);
hipError_t launch_mean_pair32(const MeanPairArgs<float>& a, hipStream_t s);

// one Lt-only sweep; out[0] = max|dLt|, out[1] = max|Lt| over the sweep (device scalars);
// partials needs 2 doubles per 256-row block
hipError_t launch_lambda_sweep(const Layout* L, const double* coef, const double* lam_in,
                               double* lam_out, double* lamout, double* partials, double* out,
                               hipStream_t s);
hipError_t launch_lambda_finalize(const Layout* L, const double* coef, const double* lam_in,
                                  Precomp* P, hipStream_t s);
// One Lt-only sweep over the lanes of colour class `colour` (-1: all, flood), in place when
// lam_in == lam_out: Sigma_j -> S[j], invS32[j]; every Lt_ji sent -> lam_out[rev p] and, at
// the sender's slot p, lamout[p] and lamout32[p]
hipError_t launch_lambda_step(const Layout* L, const double* coef, const double* lam_in,
                              double* lam_out, double* lamout, float* lamout32, double* S,
                              float* invS32, int colour, hipStream_t s);

// r = b - A_eff x_eff, x_eff = x (+ scale[0] * dx if dx); writes r (if r) and block
// partials; then reduces them into red[0..2].
// norms == false: r only (per-block partials are still written, the reduction into red is
// skipped), for callers that do not read the norms; r32 (may be null): FP32 copy of r
hipError_t launch_residual(const Layout* L, const double* coef_row, const double* b,
                           const double* x, const float* dx, const double* scale, double* r,
                           double* partials, int32_t nred, double* red, hipStream_t s,
                           bool norms = true, float* r32 = nullptr);

hipError_t launch_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t s);
// out[0] = max of partials[2q], out[1] = max of partials[2q+1] over q < nblk
hipError_t launch_max_pairs(int nblk, const double* partials, double* out, hipStream_t s);
hipError_t launch_fill64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_copy64(double* dst, const double* src, int64_t n, hipStream_t s);
// dst = (float)(src / scale[0])
hipError_t launch_cast_scaled(float* dst, const double* src, const double* scale, int64_t n,
                              hipStream_t s);
// x += scale[0] * (double)d    (scale may be null: 1)
hipError_t launch_axpy32(double* x, const float* d, const double* scale, int64_t n,
                         hipStream_t s);
hipError_t launch_axpy64(double* x, const double* d, int64_t n, hipStream_t s);
hipError_t launch_update_values(const Layout* L, const double* csr_val, int* flag,
                                hipStream_t s);
// CSR-order copy of the message state (see gabp_get_messages); lam_outgoing: lam is a
// sender-slot array (precomputed Lt), read at the reverse slot
hipError_t launch_gather_messages(const Layout* L, const double* lam, bool lam_outgoing,
                                  const double* msg, const float* msg32, double* out_lam,
                                  double* out_msg, hipStream_t s);
hipError_t launch_entry_grad(const Layout* L, const double* lam, const double* x, double* G,
                             hipStream_t s);
hipError_t launch_param_reduce(int32_t nparam, const int32_t* jptr, const int32_t* jnnz,
                               const double* jw, const double* lam, const double* x,
                               const int32_t* row, const int32_t* col, double* dtheta,
                               hipStream_t s);

// geometric multigrid (mg.cpp)
hipError_t launch_restrict_fw(int nc, const double* rf, double* bc, hipStream_t s);
hipError_t launch_prolong_add(int nc, const double* ec, double* xf, hipStream_t s);
hipError_t launch_rbgs(const Layout* L, int side, int colour, const double* b, double* x,
                       hipStream_t s);
hipError_t launch_dense_matvec(int n, const double* inv, const double* b, double* x,
                               hipStream_t s);

}  // namespace gabp
