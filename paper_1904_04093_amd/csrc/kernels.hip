// HIP kernels of libgabp for gfx950 (CDNA4).
//
// Everything here is bandwidth-bound sparse work (about 0.2-0.4 flop per byte against an
// FP64 ridge near 10 flop/byte), so there is no MFMA: the design goal is that every
// wavefront touches whole, contiguous 64-element runs of each per-slot array.
//
// Row kernels: one thread per row, 64 consecutive rows per wavefront (= one slice of the
// layout), 256 threads per block. A thread keeps its row's incoming messages in registers
// (widths up to 16 slots; a two-pass variant re-reads wider rows from cache), so the
// per-row sums of Algorithm 1 are plain in-register accumulations and no cross-lane
// traffic is needed. Reductions (residual norms, Lt convergence) go through wavefront
// shuffles and LDS in a fixed order, so repeated runs give identical bits.
#include <algorithm>
#include <cmath>

#include "gabp_internal.h"
#include "xcd.h"

namespace gabp {
namespace {

inline int nblocks(int64_t n, int b = kBlock) { return static_cast<int>((n + b - 1) / b); }

// Thread t serves lane t & 63 of slice t >> 6; that lane holds row perm[t] (-1: a padding
// lane, no row) when the context stores colour-major lanes, else row t.
__device__ __forceinline__ int row_of(const int32_t* __restrict__ perm, int t) {
  return perm ? perm[t] : t;
}

__device__ __forceinline__ int row_base(const int32_t* __restrict__ sptr, int j, int* w) {
  const int s = j >> 6;
  const int a = sptr[s];
  *w = (sptr[s + 1] - a) >> 6;
  return a + (j & 63);
}

// The same for a lane t whose whole wavefront lies in one slice (launches over lanes that
// start on a slice boundary, in workgroups of whole wavefronts): the slice index is made
// wave-uniform, so its two sptr reads are scalar loads, issued without waiting for any
// vector load (in particular not for the lane's row).
__device__ __forceinline__ int row_base_wave(const int32_t* __restrict__ sptr, int t, int* w) {
  const int s = __builtin_amdgcn_readfirstlane(t >> 6);
  const int a = sptr[s];
  *w = (sptr[s + 1] - a) >> 6;
  return a + (t & 63);
}

// ---- streaming loads/stores ----------------------------------------------------------
// Per-slot arrays are touched once per sweep and the sweep's footprint exceeds the
// last-level cache, so they are read and written with non-temporal hints.
template <bool NT, typename T>
__device__ __forceinline__ T ld_s(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p); else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_s(T v, T* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
}

// ---- wavefront / block reductions (deterministic) -------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------------------
// Joint flood sweep (Algorithm 1, FP64): read off x_j, then send Lt_ji and m_ji.
// KMAX > 0: row held in registers; KMAX == 0: two passes over memory for wide rows.
// Lanes [t0, t1): all of them (flood) or one colour class of a coloured layout, which the
// class updates in place (red-black / 4-colour schedule).
// ---------------------------------------------------------------------------------------
// Reverse slot of p: rev[p] (int32) or from the int16 delta rev16[p]: p + rev16[p] +
// rshift, where rshift is 0 for a flood layout and, for one colour class of a two-class
// layout, the distance from its first slot to the other class's; kRevSelf16 marks a padding
// slot of such a layout (its own reverse). Padding slots write zeros at themselves.
template <bool NT, bool R16>
__device__ __forceinline__ int rev_of(const int32_t* __restrict__ rev,
                                      const int16_t* __restrict__ rev16, int p, int rshift) {
  if constexpr (R16) {
    const int d = static_cast<int>(ld_s<NT>(rev16 + p));
    return d == kRevSelf16 ? p : p + d + rshift;
  } else {
    return ld_s<NT>(rev + p);
  }
}

// FIRST: the sweep right after a message reset. The incoming buffers are not read (nor
// cleared beforehand): an incoming slot counts as written only if its sender's slot rev(p)
// lies below `fresh` (the colour classes already updated in this sweep; 0 for a flood
// sweep), every other incoming message is zero.
// WX: 0 no read-off, 1 x_j = M_j / Sigma_j, 2 xadd_j += M_j / Sigma_j (the smoother's
// error correction fused into its last sweep), 3 xadd_j = M_j / Sigma_j (a smoother
// started from x = 0).
template <int KMAX, int WX, bool NT, bool R16, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_joint(
    int t1, const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const int16_t* __restrict__ rev16,
    const double* __restrict__ coef, const double* __restrict__ diag,
    const double* __restrict__ b, const double* lam_in, const double* msg_in,
    double* lam_out, double* msg_out, double* __restrict__ x, int t0, int fresh,
    const int32_t* __restrict__ perm, int rshift, double* __restrict__ xadd) {
  const int t = t0 + static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= t1) return;
  const int j = row_of(perm, t);
  int w;
  const int p0 = row_base_wave(sptr, t, &w);
  if constexpr (KMAX > 0) {
    double l[KMAX], m[KMAX], a[KMAX];
    int r[KMAX];
    // the slot loads are issued before the lane's row is known (a padding lane reads its
    // own padding slots and stops below)
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < w) {
        const int p = p0 + 64 * k;
        a[k] = ld_s<NT>(coef + p);
        r[k] = rev_of<NT, R16>(rev, rev16, p, rshift);
        if constexpr (FIRST) {
          const bool v = r[k] < fresh;
          l[k] = v ? ld_s<NT>(lam_in + p) : 0.0;
          m[k] = v ? ld_s<NT>(msg_in + p) : 0.0;
        } else {
          l[k] = ld_s<NT>(lam_in + p);
          m[k] = ld_s<NT>(msg_in + p);
        }
      }
    }
    if (j < 0) return;
    double S = diag[j];
    double M = b[j];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < w) {
        S = fma(l[k], a[k], S);
        M += m[k];
      }
    }
    if constexpr (WX == 1) x[j] = M / S;
    if constexpr (WX == 2) xadd[j] += M / S;
    if constexpr (WX == 3) xadd[j] = M / S;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < w) {
        const double L = -a[k] / (S - l[k] * a[k]);
        st_s<NT>(L, lam_out + r[k]);
        st_s<NT>(L * (M - m[k]), msg_out + r[k]);
      }
    }
  } else {
    if (j < 0) return;
    double S = diag[j];
    double M = b[j];
    auto in = [&](const double* buf, int p) -> double {
      if constexpr (FIRST) return rev_of<false, R16>(rev, rev16, p, rshift) < fresh ? buf[p] : 0.0;
      else return buf[p];
    };
    for (int k = 0; k < w; ++k) {
      const int p = p0 + 64 * k;
      S = fma(in(lam_in, p), coef[p], S);
      M += in(msg_in, p);
    }
    if constexpr (WX == 1) x[j] = M / S;
    if constexpr (WX == 2) xadd[j] += M / S;
    if constexpr (WX == 3) xadd[j] = M / S;
    for (int k = 0; k < w; ++k) {
      const int p = p0 + 64 * k;
      const double l = in(lam_in, p), a = coef[p], m = in(msg_in, p);
      const int r = rev_of<false, R16>(rev, rev16, p, rshift);
      const double L = -a / (S - l * a);
      lam_out[r] = L;
      msg_out[r] = L * (M - m);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Mean-only sweep with frozen Lt* (Sec. 2.3 decoupling, Sec. 4.2), FP64 and FP32.
// lamout[p] = Lt*_ji of the message row j sends through slot p = (j,i).
// ---------------------------------------------------------------------------------------
template <typename T>
struct ReadOff;
template <>
struct ReadOff<double> {
  static __device__ __forceinline__ double f(double M, const double* S, int j) { return M / S[j]; }
};
template <>
struct ReadOff<float> {
  static __device__ __forceinline__ float f(float M, const float* invS, int j) {
    return M * invS[j];
  }
};

template <typename T, int KMAX, int WX, bool NT, bool R16, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_mean(
    int t1, const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const int16_t* __restrict__ rev16,
    const T* __restrict__ lamout, const T* __restrict__ Sx, const T* __restrict__ b,
    const T* msg_in, T* msg_out, T* __restrict__ x, int t0, int fresh,
    const int32_t* __restrict__ perm, int rshift, double* __restrict__ xadd) {
  const int t = t0 + static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= t1) return;
  const int j = row_of(perm, t);
  int w;
  const int p0 = row_base_wave(sptr, t, &w);
  if constexpr (KMAX > 0) {
    T m[KMAX], lo[KMAX];
    int r[KMAX];
    // slot loads first, as in k_joint
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < w) {
        const int p = p0 + 64 * k;
        lo[k] = ld_s<NT>(lamout + p);
        r[k] = rev_of<NT, R16>(rev, rev16, p, rshift);
        if constexpr (FIRST) m[k] = r[k] < fresh ? ld_s<NT>(msg_in + p) : T(0);
        else m[k] = ld_s<NT>(msg_in + p);
      }
    }
    if (j < 0) return;
    T M = b[j];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < w) M += m[k];
    if constexpr (WX == 1) x[j] = ReadOff<T>::f(M, Sx, j);
    if constexpr (WX == 2) xadd[j] += static_cast<double>(ReadOff<T>::f(M, Sx, j));
    if constexpr (WX == 3) xadd[j] = static_cast<double>(ReadOff<T>::f(M, Sx, j));
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < w) st_s<NT>(lo[k] * (M - m[k]), msg_out + r[k]);
  } else {
    if (j < 0) return;
    T M = b[j];
    auto in = [&](int p) -> T {
      if constexpr (FIRST) return rev_of<false, R16>(rev, rev16, p, rshift) < fresh ? msg_in[p] : T(0);
      else return msg_in[p];
    };
    for (int k = 0; k < w; ++k) M += in(p0 + 64 * k);
    if constexpr (WX == 1) x[j] = ReadOff<T>::f(M, Sx, j);
    if constexpr (WX == 2) xadd[j] += static_cast<double>(ReadOff<T>::f(M, Sx, j));
    if constexpr (WX == 3) xadd[j] = static_cast<double>(ReadOff<T>::f(M, Sx, j));
    for (int k = 0; k < w; ++k) {
      const int p = p0 + 64 * k;
      msg_out[rev_of<false, R16>(rev, rev16, p, rshift)] = lamout[p] * (M - in(p));
    }
  }
}

// ---------------------------------------------------------------------------------------
// Two flood sweeps in one pass (temporal blocking) over a tiled layout: one workgroup per
// tile (kTileUnit slices of 64 lanes). The first kTileOwnThreads threads own the tile's
// rows, the last kHaloThreads its halo (the rows outside the tile that send into it, one
// per thread, given by {first slot, slots, row}). Sweep 1 runs for both; of the messages it sends, those into
// the tile go to LDS and the rest are dropped (the tiles they belong to compute them for
// themselves). Sweep 2 runs for the tile's rows from the LDS messages and writes its
// messages to the output buffers like a plain sweep. Same operations in the same order as
// two plain sweeps, so the results are the same bits; HBM traffic is about one sweep's plus
// the halo's.
// ---------------------------------------------------------------------------------------
// HS: cache hints of the own rows' slot streams: 0 plain, 1 non-temporal loads and stores,
// 2 non-temporal stores only (the outputs are read by the next launch, not this one; plain
// loads keep the lines a neighbouring tile's halo reads in L2)
template <int WX, int HS, bool FIRST>
__global__ __launch_bounds__(kTileThreads) void k_joint2(
    const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const int4* __restrict__ halo,
    const double* __restrict__ coef, const double* __restrict__ diag,
    const double* __restrict__ b, const double* lam_in, const double* msg_in,
    double* lam_out, double* msg_out, double* __restrict__ x,
    double* __restrict__ xadd, int slots_max, int tiles_x, int strip, int nx, int ny) {
  extern __shared__ double lds[];
  double* Ls = lds;
  double* Ms = lds + slots_max;
  const int tile = tile_of_block(blockIdx.x, gridDim.x, tiles_x, strip);
  const int ts0 = sptr[tile * kTileUnit];
  const unsigned nts = static_cast<unsigned>(sptr[(tile + 1) * kTileUnit] - ts0);
  const bool own = threadIdx.x < kTileOwnThreads;
  // own rows: coefficients, reverse slots, diagonal and b stay in registers for sweep 2
  double a[kTileMaxWidth], l[kTileMaxWidth], m[kTileMaxWidth];
  int r[kTileMaxWidth];
  int w = 0, p0 = 0, j = -1;
  double dj = 0.0, bj = 0.0;
  if (own) {
    // one slice (one grid row of 64 nodes) per own wavefront: the slot range is read with
    // scalar loads and the row follows from the tile's position, so every load of the row
    // is issued at once (a padding lane past the grid's edge reads its own padding slots
    // and row 0's entries, and sends nothing)
    const int tl = tile * kTileOwnThreads + static_cast<int>(threadIdx.x);
    p0 = row_base_wave(sptr, tl, &w);
    const int gx = (tile % tiles_x) * kSlice + (static_cast<int>(threadIdx.x) & 63);
    const int gy = (tile / tiles_x) * kTileUnit + (static_cast<int>(threadIdx.x) >> 6);
    j = gx < nx && gy < ny ? gy * nx + gx : -1;
    const int jc = j < 0 ? 0 : j;
    dj = diag[jc];
    bj = b[jc];
#pragma unroll
    for (int k = 0; k < kTileMaxWidth; ++k) {
      if (k < w) {
        const int p = p0 + 64 * k;
        a[k] = ld_s<HS == 1>(coef + p);
        r[k] = ld_s<HS == 1>(rev + p);
        l[k] = FIRST ? 0.0 : ld_s<HS == 1>(lam_in + p);
        m[k] = FIRST ? 0.0 : ld_s<HS == 1>(msg_in + p);
      }
    }
  }
  // sweep 1: own rows (every message into the tile) and halo rows (their messages into it)
  auto send1 = [&](int wd, double S, double M) {
#pragma unroll
    for (int k = 0; k < kTileMaxWidth; ++k) {
      const unsigned q = static_cast<unsigned>(r[k] - ts0);
      if (k < wd && q < nts) {
        const double L = -a[k] / (S - l[k] * a[k]);
        Ls[q] = L;
        Ms[q] = L * (M - m[k]);
      }
    }
  };
  if (own) {
    if (j >= 0) {
      double S = dj, M = bj;
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        if (k < w) {
          S = fma(l[k], a[k], S);
          M += m[k];
        }
      }
      send1(w, S, M);
    }
  } else {
    // one halo row per halo thread (entries past the tile's halo have no slots)
    const int4 h = halo[tile * kHaloThreads + static_cast<int>(threadIdx.x) - kTileOwnThreads];
    if (h.y > 0) {   // {first slot, slots, row, -}
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        if (k < h.y) {
          const int p = h.x + 64 * k;
          a[k] = coef[p];
          r[k] = rev[p];
          l[k] = FIRST ? 0.0 : lam_in[p];
          m[k] = FIRST ? 0.0 : msg_in[p];
        }
      }
      double S = diag[h.z], M = b[h.z];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        if (k < h.y) {
          S = fma(l[k], a[k], S);
          M += m[k];
        }
      }
      send1(h.y, S, M);
    }
  }
  __syncthreads();
  if (j < 0) return;
  // sweep 2 of the own rows, from the LDS messages
  double S = dj, M = bj;
#pragma unroll
  for (int k = 0; k < kTileMaxWidth; ++k) {
    if (k < w) {
      const int q = p0 + 64 * k - ts0;
      l[k] = Ls[q];
      m[k] = Ms[q];
      S = fma(l[k], a[k], S);
      M += m[k];
    }
  }
  if constexpr (WX == 1) x[j] = M / S;
  if constexpr (WX == 2) xadd[j] += M / S;
  if constexpr (WX == 3) xadd[j] = M / S;
#pragma unroll
  for (int k = 0; k < kTileMaxWidth; ++k) {
    if (k < w) {
      const double L = -a[k] / (S - l[k] * a[k]);
      st_s<HS != 0>(L, lam_out + r[k]);
      st_s<HS != 0>(L * (M - m[k]), msg_out + r[k]);
    }
  }
}

// Mean-only form (frozen or per-sweep precomputed Lt): sweep 1 sends with lamA, sweep 2
// reads off with SxB (Sigma, or 1/Sigma for FP32) and sends with lamB. Tiles of TS slices:
// each own thread takes TS / kTileUnit lanes, kTileOwnThreads apart.
template <typename T, int TS, int WX, int HS, bool FIRST>
__global__ __launch_bounds__(kTileThreads) void k_mean2(
    const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const int4* __restrict__ halo,
    const T* __restrict__ lamA, const T* __restrict__ lamB, const T* __restrict__ SxB,
    const T* __restrict__ b, const T* msg_in, T* msg_out, T* __restrict__ x,
    double* __restrict__ xadd, int tiles_x, int strip, int nx, int ny) {
  constexpr int RPT = TS / kTileUnit;
  extern __shared__ double lds_raw[];
  T* Ms = reinterpret_cast<T*>(lds_raw);
  const int tile = tile_of_block(blockIdx.x, gridDim.x, tiles_x, strip);
  const int ts0 = sptr[tile * TS];
  const unsigned nts = static_cast<unsigned>(sptr[(tile + 1) * TS] - ts0);
  const bool own = threadIdx.x < kTileOwnThreads;
  T lb[RPT][kTileMaxWidth], m[RPT][kTileMaxWidth];
  int r[RPT][kTileMaxWidth];
  int w[RPT], p0[RPT], j[RPT];
  T bj[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    j[q] = -1;
    w[q] = 0;
    p0[q] = 0;
  }
  if (own) {
    // every load of the thread's lanes first, then the sends
    T lo[RPT][kTileMaxWidth];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      // as in k_joint2: scalar slot range per wavefront, the row from the tile's position
      const int tl = tile * TS * kSlice + static_cast<int>(threadIdx.x) + q * kTileOwnThreads;
      p0[q] = row_base_wave(sptr, tl, &w[q]);
      const int gx = (tile % tiles_x) * kSlice + (static_cast<int>(threadIdx.x) & 63);
      const int gy = (tile / tiles_x) * TS + (static_cast<int>(threadIdx.x) >> 6) + q * kTileUnit;
      j[q] = gx < nx && gy < ny ? gy * nx + gx : -1;
      bj[q] = b[j[q] < 0 ? 0 : j[q]];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        if (k < w[q]) {
          const int p = p0[q] + 64 * k;
          lo[q][k] = ld_s<HS == 1>(lamA + p);
          lb[q][k] = lamB == lamA ? lo[q][k] : ld_s<HS == 1>(lamB + p);
          r[q][k] = ld_s<HS == 1>(rev + p);
          m[q][k] = FIRST ? T(0) : ld_s<HS == 1>(msg_in + p);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (j[q] < 0) continue;
      T M = bj[q];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k)
        if (k < w[q]) M += m[q][k];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        const unsigned qq = static_cast<unsigned>(r[q][k] - ts0);
        if (k < w[q] && qq < nts) Ms[qq] = lo[q][k] * (M - m[q][k]);
      }
    }
  } else {
    const int4 h = halo[tile * kHaloThreads + static_cast<int>(threadIdx.x) - kTileOwnThreads];
    if (h.y > 0) {   // {first slot, slots, row, -}
      T loh[kTileMaxWidth], mh[kTileMaxWidth];
      int rh[kTileMaxWidth];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        if (k < h.y) {
          const int p = h.x + 64 * k;
          loh[k] = lamA[p];
          rh[k] = rev[p];
          mh[k] = FIRST ? T(0) : msg_in[p];
        }
      }
      T M = b[h.z];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k)
        if (k < h.y) M += mh[k];
#pragma unroll
      for (int k = 0; k < kTileMaxWidth; ++k) {
        const unsigned qq = static_cast<unsigned>(rh[k] - ts0);
        if (k < h.y && qq < nts) Ms[qq] = loh[k] * (M - mh[k]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    if (j[q] < 0) continue;
    T M = bj[q];
#pragma unroll
    for (int k = 0; k < kTileMaxWidth; ++k) {
      if (k < w[q]) {
        m[q][k] = Ms[p0[q] + 64 * k - ts0];
        M += m[q][k];
      }
    }
    if constexpr (WX == 1) x[j[q]] = ReadOff<T>::f(M, SxB, j[q]);
    if constexpr (WX == 2) xadd[j[q]] += static_cast<double>(ReadOff<T>::f(M, SxB, j[q]));
    if constexpr (WX == 3) xadd[j[q]] = static_cast<double>(ReadOff<T>::f(M, SxB, j[q]));
#pragma unroll
    for (int k = 0; k < kTileMaxWidth; ++k)
      if (k < w[q]) st_s<HS != 0>(lb[q][k] * (M - m[q][k]), msg_out + r[q][k]);
  }
}

// ---------------------------------------------------------------------------------------
// Lt-only flood sweep for the precompute phase. Also records the outgoing value at the
// sender's own slot (lamout) and the largest change / magnitude of this sweep.
// ---------------------------------------------------------------------------------------
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_lambda(
    int n, const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const double* __restrict__ coef, const double* __restrict__ diag, const double* lam_in,
    double* lam_out, double* __restrict__ lamout, double* __restrict__ partials,
    const int32_t* __restrict__ perm) {
  __shared__ double sh[2][kBlock / 64];
  const int t = blockIdx.x * kBlock + threadIdx.x;
  double dm = 0.0, lm = 0.0;
  const int j = t < n ? row_of(perm, t) : -1;   // n: lanes
  if (j >= 0) {
    int w;
    const int p0 = row_base(sptr, t, &w);
    double S = diag[j];
    if constexpr (KMAX > 0) {
      double l[KMAX], a[KMAX];
      int r[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < w) {
          const int p = p0 + 64 * k;
          l[k] = lam_in[p];
          a[k] = coef[p];
          r[k] = rev[p];
        }
      }
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k < w) S = fma(l[k], a[k], S);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < w) {
          const int p = p0 + 64 * k;
          const double L = -a[k] / (S - l[k] * a[k]);
          dm = fmax(dm, fabs(L - lamout[p]));
          lm = fmax(lm, fabs(L));
          lamout[p] = L;
          lam_out[r[k]] = L;
        }
      }
    } else {
      for (int k = 0; k < w; ++k) {
        const int p = p0 + 64 * k;
        S = fma(lam_in[p], coef[p], S);
      }
      for (int k = 0; k < w; ++k) {
        const int p = p0 + 64 * k;
        const double l = lam_in[p], a = coef[p];
        const double L = -a / (S - l * a);
        dm = fmax(dm, fabs(L - lamout[p]));
        lm = fmax(lm, fabs(L));
        lamout[p] = L;
        lam_out[rev[p]] = L;
      }
    }
  }
  // NaN anywhere must stop the phase: map it to +inf for the ordered-bits maximum
  if (dm != dm) dm = INFINITY;
  if (lm != lm) lm = INFINITY;
  dm = wave_max(dm);
  lm = wave_max(lm);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = dm;
    sh[1][wv] = lm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double d2 = sh[0][0], l2 = sh[1][0];
    for (int q = 1; q < kBlock / 64; ++q) {
      d2 = fmax(d2, sh[0][q]);
      l2 = fmax(l2, sh[1][q]);
    }
    partials[2 * blockIdx.x + 0] = d2;
    partials[2 * blockIdx.x + 1] = l2;
  }
}

// max over the per-block partials of k_lambda -> out[0] = max|dLt|, out[1] = max|Lt|
__global__ __launch_bounds__(1024) void k_lambda_reduce(int nblk, const double* __restrict__ partials,
                                                        double* __restrict__ out) {
  __shared__ double sh[2][16];
  double d = 0.0, l = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 1024) {
    d = fmax(d, partials[2 * q]);
    l = fmax(l, partials[2 * q + 1]);
  }
  d = wave_max(d);
  l = wave_max(l);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = d;
    sh[1][threadIdx.x >> 6] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 16; ++q) {
      d = fmax(d, sh[0][q]);
      l = fmax(l, sh[1][q]);
    }
    d = fmax(d, sh[0][0]);
    l = fmax(l, sh[1][0]);
    out[0] = d;
    out[1] = l;
  }
}


template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_lambda_fin(
    int n, const int32_t* __restrict__ sptr, const double* __restrict__ coef,
    const double* __restrict__ diag, const double* __restrict__ lam_in,
    const double* __restrict__ lamout, double* __restrict__ Sout, float* __restrict__ lamout32,
    float* __restrict__ invS32, const int32_t* __restrict__ perm) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;   // n: lanes
  const int j = row_of(perm, t);
  if (j < 0) return;
  int w;
  const int p0 = row_base(sptr, t, &w);
  double S = diag[j];
  for (int k = 0; k < w; ++k) {
    const int p = p0 + 64 * k;
    S = fma(lam_in[p], coef[p], S);
    lamout32[p] = static_cast<float>(lamout[p]);
  }
  Sout[j] = S;
  invS32[j] = static_cast<float>(1.0 / S);
}

// One Lt-only sweep that keeps what it computes: the node precisions of this sweep's
// read-off and the messages it sends, at the sender's slot (per-sweep precompute). Lanes
// [t0, t1): all (flood, lam_in != lam_out) or one colour class (in place). Runs once per
// matrix, so it is the plain two-pass form.
__global__ __launch_bounds__(kBlock) void k_lambda_step(
    int t1, const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const double* __restrict__ coef, const double* __restrict__ diag, const double* lam_in,
    double* lam_out, double* __restrict__ lamout, float* __restrict__ lamout32,
    double* __restrict__ Sout, float* __restrict__ invS32, int t0,
    const int32_t* __restrict__ perm) {
  const int t = t0 + static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
  if (t >= t1) return;
  const int j = row_of(perm, t);
  if (j < 0) return;
  int w;
  const int p0 = row_base(sptr, t, &w);
  double S = diag[j];
  for (int k = 0; k < w; ++k) {
    const int p = p0 + 64 * k;
    S = fma(lam_in[p], coef[p], S);
  }
  Sout[j] = S;
  invS32[j] = static_cast<float>(1.0 / S);
  for (int k = 0; k < w; ++k) {
    const int p = p0 + 64 * k;
    const double l = lam_in[p], a = coef[p];
    const double L = -a / (S - l * a);
    lamout[p] = L;
    lamout32[p] = static_cast<float>(L);
    lam_out[rev[p]] = L;
  }
}

// ---------------------------------------------------------------------------------------
// Residual r = b - A x (coef_row = val) or b - A^T x (coef_row = aT), optionally at
// x + scale * dx, with per-block partial norms. Threads take rows in row order, also for a
// colour-major layout (a row's slots found through its lane), so that b, x, diag and r are
// read and written in whole runs and a row's neighbours are gathered near its own x. NT:
// the streamed inputs (row slots, b, diag, columns, coefficients) with non-temporal loads,
// x (gathered by the neighbouring rows) with plain ones.
// ---------------------------------------------------------------------------------------
template <int KMAX, bool XADD, bool NT>
__global__ __launch_bounds__(kRedBlock) void k_residual(
    int n, const int32_t* __restrict__ sptr, const int32_t* __restrict__ col,
    const double* __restrict__ coef_row, const double* __restrict__ diag,
    const double* __restrict__ b, const double* __restrict__ x, const float* __restrict__ dx,
    const double* __restrict__ scale, double* __restrict__ r, double* __restrict__ partials,
    const int32_t* __restrict__ lane_of_row, float* __restrict__ r32,
    const int32_t* __restrict__ row_slot) {
  __shared__ double sh[3][kRedBlock / 64];
  const int blk = xcd_block(blockIdx.x, gridDim.x);   // row range and partials slot
  const int t = blk * kRedBlock + threadIdx.x;
  double rr = 0.0, ra = 0.0, bb = 0.0;
  const int j = t < n ? t : -1;   // n: rows
  if (j >= 0) {
    int w, p0;
    if (row_slot) {   // first slot and slice width of row j, packed: one load, no sptr
      const unsigned v = static_cast<unsigned>(ld_s<NT>(row_slot + j));
      p0 = static_cast<int>(v & kRowSlotMask);
      w = static_cast<int>(v >> kRowSlotShift);
    } else {
      p0 = row_base(sptr, lane_of_row ? lane_of_row[j] : j, &w);
    }
    const double sc = XADD ? scale[0] : 0.0;
    double xj = x[j];
    if (XADD) xj = fma(sc, static_cast<double>(dx[j]), xj);
    const double bj = ld_s<NT>(b + j);
    double acc = fma(-ld_s<NT>(diag + j), xj, bj);
    if constexpr (KMAX > 0) {
      // all index and coefficient loads first, then the gathers: more bytes in flight
      int cc[KMAX];
      double cf[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < w) {
          cc[k] = ld_s<NT>(col + p0 + 64 * k);
          cf[k] = ld_s<NT>(coef_row + p0 + 64 * k);
        }
      }
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < w) {
          double xc = x[cc[k]];
          if (XADD) xc = fma(sc, static_cast<double>(dx[cc[k]]), xc);
          acc = fma(-cf[k], xc, acc);
        }
      }
    } else {
      for (int k = 0; k < w; ++k) {
        const int p = p0 + 64 * k;
        const int cc = col[p];
        double xc = x[cc];
        if (XADD) xc = fma(sc, static_cast<double>(dx[cc]), xc);
        acc = fma(-coef_row[p], xc, acc);
      }
    }
    if (r) r[j] = acc;
    if (r32) r32[j] = static_cast<float>(acc);
    rr = acc * acc;
    ra = fabs(acc);
    if (ra != ra) ra = INFINITY;
    bb = bj * bj;
  }
  rr = wave_sum(rr);
  ra = wave_max(ra);
  bb = wave_sum(bb);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = rr;
    sh[1][wv] = ra;
    sh[2][wv] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = sh[0][0], s1 = sh[1][0], s2 = sh[2][0];
    for (int q = 1; q < kRedBlock / 64; ++q) {
      s0 += sh[0][q];
      s1 = fmax(s1, sh[1][q]);
      s2 += sh[2][q];
    }
    partials[3 * blk + 0] = s0;
    partials[3 * blk + 1] = s1;
    partials[3 * blk + 2] = s2;
  }
}

// Plain streaming copy: one 16-byte vector per thread with non-temporal hints, the fastest
// of the copy shapes tried on gfx950 (grid-stride loops reach ~25% less).
typedef double v2d __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_copy_probe(const v2d* __restrict__ src,
                                                   v2d* __restrict__ dst, int64_t n2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n2) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

constexpr int kFinBlock = 1024;
__global__ __launch_bounds__(kFinBlock) void k_finalize_norms(
    int nred, const double* __restrict__ partials, double* __restrict__ red) {
  __shared__ double sh[3][kFinBlock / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int q = threadIdx.x; q < nred; q += kFinBlock) {
    s0 += partials[3 * q + 0];
    s1 = fmax(s1, partials[3 * q + 1]);
    s2 += partials[3 * q + 2];
  }
  s0 = wave_sum(s0);
  s1 = wave_max(s1);
  s2 = wave_sum(s2);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = s0;
    sh[1][wv] = s1;
    sh[2][wv] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = sh[0][0], t1 = sh[1][0], t2 = sh[2][0];
    for (int q = 1; q < kFinBlock / 64; ++q) {
      t0 += sh[0][q];
      t1 = fmax(t1, sh[1][q]);
      t2 += sh[2][q];
    }
    red[0] = t0;
    red[1] = t1;
    red[2] = t2;
    red[3] = t1;  // max|r|: the scale used by iterative refinement
  }
}

// ---- elementwise helpers --------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_copy64(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
__global__ void k_cast_scaled(float* __restrict__ d, const double* __restrict__ s,
                              const double* __restrict__ scale, int64_t n) {
  const double inv = scale ? 1.0 / scale[0] : 1.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = static_cast<float>(s[i] * inv);
}
__global__ void k_axpy32(double* __restrict__ x, const float* __restrict__ d,
                         const double* __restrict__ scale, int64_t n) {
  const double sc = scale ? scale[0] : 1.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = fma(sc, static_cast<double>(d[i]), x[i]);
}
__global__ void k_axpy64(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += d[i];
}

__global__ void k_update_slots(int64_t epad, const int32_t* __restrict__ vsrc,
                               const int32_t* __restrict__ asrc, const double* __restrict__ csr,
                               double* __restrict__ val, double* __restrict__ aT) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < epad;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = vsrc[p], a = asrc[p];
    val[p] = v >= 0 ? csr[v] : 0.0;
    aT[p] = a >= 0 ? csr[a] : 0.0;
  }
}
__global__ void k_update_diag(int n, const int32_t* __restrict__ dsrc,
                              const double* __restrict__ csr, double* __restrict__ diag,
                              int* __restrict__ bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double d = csr[dsrc[j]];
  diag[j] = d;
  if (!(d != 0.0) || !isfinite(d)) atomicOr(bad, 1);
}

// Message state in setup CSR order: slot p = (j,i) holds the message i -> j, which belongs
// to CSR entry (j,i) = val_src[p]. lam_outgoing: lam holds the sender-slot copy of the
// precomputed Lt (the value at p is the one j sends), so the incoming one is lam[rev p].
__global__ void k_gather_messages(int64_t epad, const int32_t* __restrict__ vsrc,
                                  const int32_t* __restrict__ rev, const double* __restrict__ lam,
                                  int lam_outgoing, const double* __restrict__ msg,
                                  const float* __restrict__ msg32, double* __restrict__ out_lam,
                                  double* __restrict__ out_msg) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < epad;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = vsrc[p];
    if (e < 0) continue;
    if (out_lam) out_lam[e] = lam ? (lam_outgoing ? lam[rev[p]] : lam[p]) : 0.0;
    if (out_msg) out_msg[e] = msg ? msg[p] : (msg32 ? static_cast<double>(msg32[p]) : 0.0);
  }
}

__global__ void k_entry_grad(int64_t nnz, const int32_t* __restrict__ row,
                             const int32_t* __restrict__ col, const double* __restrict__ lam,
                             const double* __restrict__ x, double* __restrict__ G) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    G[e] = -lam[row[e]] * x[col[e]];
}
__global__ void k_param_reduce(int np, const int32_t* __restrict__ jptr,
                               const int32_t* __restrict__ jnnz, const double* __restrict__ jw,
                               const double* __restrict__ lam, const double* __restrict__ x,
                               const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                               double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double acc = 0.0;
  for (int k = jptr[p]; k < jptr[p + 1]; ++k) {
    const int e = jnnz[k];
    acc = fma(jw[k], -lam[row[e]] * x[col[e]], acc);
  }
  out[p] = acc;
}

// ---- geometric multigrid on vertex-centred n x n interior grids (x fastest) ------------
// Full weighting: b_c(I,J) = [1 2 1; 2 4 2; 1 2 1] / 16 around fine node (2I+1, 2J+1).
__global__ void k_restrict_fw(int nc, const double* __restrict__ rf, double* __restrict__ bc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc * nc) return;
  const int nf = 2 * nc + 1;
  const int I = q % nc, J = q / nc;
  const int fx = 2 * I + 1, fy = 2 * J + 1;
  const double* c = rf + (int64_t)fy * nf + fx;
  const double centre = c[0];
  const double edges = c[-1] + c[1] + c[-nf] + c[nf];
  const double corners = c[-nf - 1] + c[-nf + 1] + c[nf - 1] + c[nf + 1];
  bc[q] = (4.0 * centre + 2.0 * edges + corners) * (1.0 / 16.0);
}

// Bilinear interpolation of the coarse correction (zero on the boundary), added to x_f.
__device__ __forceinline__ double coarse_at(const double* ec, int nc, int cx, int cy) {
  // cx, cy: coarse indices including the boundary ring (0 and nc + 1 are boundary)
  return (cx < 1 || cy < 1 || cx > nc || cy > nc) ? 0.0 : ec[(int64_t)(cy - 1) * nc + (cx - 1)];
}
__global__ void k_prolong_add(int nc, const double* __restrict__ ec, double* __restrict__ xf) {
  const int nf = 2 * nc + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nf * nf) return;
  const int Fx = q % nf + 1, Fy = q / nf + 1;   // fine indices including the boundary ring
  double v;
  if ((Fy & 1) == 0) {
    if ((Fx & 1) == 0) v = coarse_at(ec, nc, Fx / 2, Fy / 2);
    else v = 0.5 * (coarse_at(ec, nc, Fx / 2, Fy / 2) + coarse_at(ec, nc, Fx / 2 + 1, Fy / 2));
  } else {
    double lo, hi;
    if ((Fx & 1) == 0) {
      lo = coarse_at(ec, nc, Fx / 2, Fy / 2);
      hi = coarse_at(ec, nc, Fx / 2, Fy / 2 + 1);
    } else {
      lo = 0.5 * (coarse_at(ec, nc, Fx / 2, Fy / 2) + coarse_at(ec, nc, Fx / 2 + 1, Fy / 2));
      hi = 0.5 * (coarse_at(ec, nc, Fx / 2, Fy / 2 + 1) + coarse_at(ec, nc, Fx / 2 + 1, Fy / 2 + 1));
    }
    v = 0.5 * (lo + hi);
  }
  xf[q] += v;
}

// One colour of red-black Gauss-Seidel: x_j = (b_j - sum_{k != j} A_jk x_k) / A_jj for the
// rows with (ix + iy) % 2 == c, in place (the 5-point graph is bipartite in this colouring).
template <int KMAX>
__global__ __launch_bounds__(kBlock) void k_rbgs(int n, int side, int c,
                                                 const int32_t* __restrict__ sptr,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ diag,
                                                 const double* __restrict__ b, double* x,
                                                 const int32_t* __restrict__ perm) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;   // n: lanes
  const int j = row_of(perm, t);
  if (j < 0 || ((j % side) + (j / side)) % 2 != c) return;
  int w;
  const int p0 = row_base(sptr, t, &w);
  double s = 0.0;
  for (int k = 0; k < w; ++k) {
    const int p = p0 + 64 * k;
    s = fma(val[p], x[col[p]], s);
  }
  x[j] = (b[j] - s) / diag[j];
}

// Coarsest level: x = A^{-1} b with the inverse formed once on the host.
__global__ void k_dense_matvec(int n, const double* __restrict__ inv, const double* __restrict__ b,
                               double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc = fma(inv[(int64_t)i * n + k], b[k], acc);
  x[i] = acc;
}

int grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return static_cast<int>(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

}  // namespace

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
#define GABP_DISPATCH_WIDTH(W, CALL4, CALL8, CALL16, CALL0) \
  do {                                                      \
    if ((W) <= 4) { CALL4; }                                \
    else if ((W) <= 8) { CALL8; }                           \
    else if ((W) <= 16) { CALL16; }                         \
    else { CALL0; }                                         \
  } while (0)

#define GABP_DISPATCH_NT(NTV, ...)                   \
  if (NTV) { constexpr bool NTB = true; __VA_ARGS__; } \
  else { constexpr bool NTB = false; __VA_ARGS__; }
#define GABP_DISPATCH_HS(HV, ...)                                    \
  if ((HV) == 2) { constexpr int HSB = 2; __VA_ARGS__; }             \
  else if ((HV) == 1) { constexpr int HSB = 1; __VA_ARGS__; }        \
  else { constexpr int HSB = 0; __VA_ARGS__; }
#define GABP_DISPATCH_R16(RV, ...)                     \
  if (RV) { constexpr bool R16B = true; __VA_ARGS__; } \
  else { constexpr bool R16B = false; __VA_ARGS__; }
#define GABP_DISPATCH_FIRST(FV, ...)                    \
  if (FV) { constexpr bool FB = true; __VA_ARGS__; }  \
  else { constexpr bool FB = false; __VA_ARGS__; }
#define GABP_DISPATCH_WX(WV, ...)                                    \
  if ((WV) == 3) { constexpr int WXB = 3; __VA_ARGS__; }             \
  else if ((WV) == 2) { constexpr int WXB = 2; __VA_ARGS__; }        \
  else if ((WV) == 1) { constexpr int WXB = 1; __VA_ARGS__; }        \
  else { constexpr int WXB = 0; __VA_ARGS__; }

// Whether a sweep over colour class c (-1: all lanes) reads the int16 reverse deltas, and
// the shift they are taken from: a flood sweep over a classed layout reads rev instead.
inline bool use_rev16(const Layout& L, int c, int* rshift) {
  *rshift = 0;
  if (!L.rev16) return false;
  if (!L.rev16_classed) return true;
  if (c < 0 || L.cslot.size() != 3) return false;
  *rshift = L.cslot[1 - c] - L.cslot[c];
  return true;
}

// lanes of a sweep: all, or those of colour class c
inline void lane_range(const Layout& L, int c, int* t0, int* t1) {
  *t0 = c >= 0 ? L.cstart[c] : 0;
  *t1 = c >= 0 ? L.cstart[c + 1] : L.nlanes;
}

hipError_t launch_joint_sweep(const SweepArgs& a, hipStream_t s) {
  const Layout& L = *a.L;
  int t0, t1;
  lane_range(L, a.colour, &t0, &t1);
  if (t1 <= t0) return hipSuccess;
  const int blk = L.block;
  const int g = nblocks(t1 - t0, blk);
#define JOINT_ARGS                                                                      \
  t1, L.sptr, L.rev, L.rev16, a.coef, L.diag, a.b, a.lam_in, a.msg_in, a.lam_out,        \
      a.msg_out, a.x, t0, a.fresh, L.perm, rshift, a.xadd
  int rshift;
  const bool r16 = use_rev16(L, a.colour, &rshift);
  GABP_DISPATCH_FIRST(a.fresh >= 0, GABP_DISPATCH_NT(L.stream_hints, GABP_DISPATCH_R16(r16,
    GABP_DISPATCH_WX(a.xadd ? (a.xset ? 3 : 2) : (a.x ? 1 : 0), {
      GABP_DISPATCH_WIDTH(L.max_width,
                          (k_joint<4, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(JOINT_ARGS)),
                          (k_joint<8, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(JOINT_ARGS)),
                          (k_joint<16, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(JOINT_ARGS)),
                          (k_joint<0, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(JOINT_ARGS)));
    }))))
#undef JOINT_ARGS
  return hipGetLastError();
}

template <typename T, typename A>
hipError_t mean_dispatch(const Layout& L, const A& a, const T* Sx, bool nt, hipStream_t s) {
  int t0, t1;
  lane_range(L, a.colour, &t0, &t1);
  if (t1 <= t0) return hipSuccess;
  const int blk = L.block;
  const int g = nblocks(t1 - t0, blk);
#define MEAN_ARGS \
  t1, L.sptr, L.rev, L.rev16, a.lamout, Sx, a.b, a.msg_in, a.msg_out, a.x, t0, a.fresh, L.perm, \
      rshift, a.xadd
  int rshift;
  const bool r16 = use_rev16(L, a.colour, &rshift);
  GABP_DISPATCH_FIRST(a.fresh >= 0, GABP_DISPATCH_NT(nt, GABP_DISPATCH_R16(r16,
    GABP_DISPATCH_WX(a.xadd ? (a.xset ? 3 : 2) : (a.x ? 1 : 0), {
      GABP_DISPATCH_WIDTH(L.max_width,
                          (k_mean<T, 4, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(MEAN_ARGS)),
                          (k_mean<T, 8, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(MEAN_ARGS)),
                          (k_mean<T, 16, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(MEAN_ARGS)),
                          (k_mean<T, 0, WXB, NTB, R16B, FB><<<g, blk, 0, s>>>(MEAN_ARGS)));
    }))))
#undef MEAN_ARGS
  return hipGetLastError();
}

hipError_t launch_joint_pair(const SweepArgs& a, hipStream_t s) {
  const Layout& L = *a.L;
  if (L.ntiles <= 0 || L.tile_slices != kTileUnit) return hipErrorInvalidValue;
  const size_t lds = 2 * static_cast<size_t>(L.tile_slots_max) * sizeof(double);
#define JOINT2_ARGS                                                                         \
  L.sptr, L.rev, L.tile_halo, a.coef, L.diag, a.b, a.lam_in, a.msg_in,          \
      a.lam_out, a.msg_out, a.x, a.xadd, L.tile_slots_max, L.tiles_x, L.tile_strip, L.grid_nx, \
      L.grid_ny
  const int hs = L.stream_hints ? 1 : (L.store_hints ? 2 : 0);
  GABP_DISPATCH_FIRST(a.fresh >= 0, GABP_DISPATCH_HS(hs,
    GABP_DISPATCH_WX(a.xadd ? (a.xset ? 3 : 2) : (a.x ? 1 : 0), {
      k_joint2<WXB, HSB, FB><<<L.ntiles, kTileThreads, lds, s>>>(JOINT2_ARGS);
    })))
#undef JOINT2_ARGS
  return hipGetLastError();
}

template <typename T>
hipError_t mean_pair_dispatch(const MeanPairArgs<T>& a, int hs, hipStream_t s) {
  const Layout& L = *a.L;
  if (L.ntiles <= 0) return hipErrorInvalidValue;
  const size_t lds = static_cast<size_t>(L.tile_slots_max) * sizeof(T);
#define MEAN2_ARGS                                                                          \
  L.sptr, L.rev, L.tile_halo, a.lamA, a.lamB, a.SxB, a.b, a.msg_in, a.msg_out,  \
      a.x, a.xadd, L.tiles_x, L.tile_strip, L.grid_nx, L.grid_ny
  GABP_DISPATCH_FIRST(a.fresh >= 0, GABP_DISPATCH_HS(hs,
    GABP_DISPATCH_WX(a.xadd ? (a.xset ? 3 : 2) : (a.x ? 1 : 0), {
      if (L.tile_slices == 2 * kTileUnit)
        k_mean2<T, 2 * kTileUnit, WXB, HSB, FB><<<L.ntiles, kTileThreads, lds, s>>>(MEAN2_ARGS);
      else
        k_mean2<T, kTileUnit, WXB, HSB, FB><<<L.ntiles, kTileThreads, lds, s>>>(MEAN2_ARGS);
    })))
#undef MEAN2_ARGS
  return hipGetLastError();
}

hipError_t launch_mean_pair64(const MeanPairArgs<double>& a, hipStream_t s) {
  const Layout& L = *a.L;
  return mean_pair_dispatch<double>(a, L.stream_hints ? 1 : (L.store_hints ? 2 : 0), s);
}

hipError_t launch_mean_pair32(const MeanPairArgs<float>& a, hipStream_t s) {
  const Layout& L = *a.L;
  return mean_pair_dispatch<float>(a, L.stream_hints32 ? 1 : (L.store_hints32 ? 2 : 0), s);
}

hipError_t launch_mean_sweep64(const MeanArgs64& a, hipStream_t s) {
  return mean_dispatch<double>(*a.L, a, a.S, a.L->stream_hints, s);
}

hipError_t launch_mean_sweep32(const MeanArgs32& a, hipStream_t s) {
  return mean_dispatch<float>(*a.L, a, a.invS, a.L->stream_hints32, s);
}

hipError_t launch_lambda_sweep(const Layout* Lp, const double* coef, const double* lam_in,
                               double* lam_out, double* lamout, double* partials, double* out,
                               hipStream_t s) {
  const Layout& L = *Lp;
  const int g = nblocks(L.nlanes);
  GABP_DISPATCH_WIDTH(
      L.max_width,
      (k_lambda<4><<<g, kBlock, 0, s>>>(L.nlanes, L.sptr, L.rev, coef, L.diag, lam_in, lam_out, lamout, partials, L.perm)),
      (k_lambda<8><<<g, kBlock, 0, s>>>(L.nlanes, L.sptr, L.rev, coef, L.diag, lam_in, lam_out, lamout, partials, L.perm)),
      (k_lambda<16><<<g, kBlock, 0, s>>>(L.nlanes, L.sptr, L.rev, coef, L.diag, lam_in, lam_out, lamout, partials, L.perm)),
      (k_lambda<0><<<g, kBlock, 0, s>>>(L.nlanes, L.sptr, L.rev, coef, L.diag, lam_in, lam_out, lamout, partials, L.perm)));
  k_lambda_reduce<<<1, 1024, 0, s>>>(g, partials, out);
  return hipGetLastError();
}

hipError_t launch_max_pairs(int nblk, const double* partials, double* out, hipStream_t s) {
  k_lambda_reduce<<<1, 1024, 0, s>>>(nblk, partials, out);
  return hipGetLastError();
}

hipError_t launch_lambda_finalize(const Layout* Lp, const double* coef, const double* lam_in,
                                  Precomp* P, hipStream_t s) {
  const Layout& L = *Lp;
  k_lambda_fin<0><<<nblocks(L.nlanes), kBlock, 0, s>>>(L.nlanes, L.sptr, coef, L.diag, lam_in,
                                                  P->lamout, P->S, P->lamout32, P->invS32,
                                                  L.perm);
  return hipGetLastError();
}

hipError_t launch_lambda_step(const Layout* Lp, const double* coef, const double* lam_in,
                              double* lam_out, double* lamout, float* lamout32, double* S,
                              float* invS32, int colour, hipStream_t s) {
  const Layout& L = *Lp;
  int t0, t1;
  lane_range(L, colour, &t0, &t1);
  if (t1 <= t0) return hipSuccess;
  k_lambda_step<<<nblocks(t1 - t0), kBlock, 0, s>>>(t1, L.sptr, L.rev, coef, L.diag, lam_in,
                                                    lam_out, lamout, lamout32, S, invS32, t0,
                                                    L.perm);
  return hipGetLastError();
}

hipError_t launch_residual(const Layout* Lp, const double* coef_row, const double* b,
                           const double* x, const float* dx, const double* scale, double* r,
                           double* partials, int32_t nred, double* red, hipStream_t s,
                           bool norms, float* r32) {
  const Layout& L = *Lp;
#define RES_ARGS(DX, SC) \
  L.n, L.sptr, L.col, coef_row, L.diag, b, x, DX, SC, r, partials, L.lane_of_row_d, r32, L.row_slot
  GABP_DISPATCH_NT(L.res_hints, {
    if (dx) {
      GABP_DISPATCH_WIDTH(L.max_width,
                          (k_residual<4, true, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(dx, scale))),
                          (k_residual<8, true, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(dx, scale))),
                          (k_residual<16, true, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(dx, scale))),
                          (k_residual<0, true, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(dx, scale))));
    } else {
      GABP_DISPATCH_WIDTH(L.max_width,
                          (k_residual<4, false, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(nullptr, nullptr))),
                          (k_residual<8, false, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(nullptr, nullptr))),
                          (k_residual<16, false, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(nullptr, nullptr))),
                          (k_residual<0, false, NTB><<<nred, kRedBlock, 0, s>>>(RES_ARGS(nullptr, nullptr))));
    }
  })
#undef RES_ARGS
  if (norms) k_finalize_norms<<<1, kFinBlock, 0, s>>>(nred, partials, red);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t n2 = bytes / 16;
  for (int64_t off = 0; off < n2;) {   // grids of at most 2^31 - 1 threads
    const int64_t chunk = std::min<int64_t>(n2 - off, int64_t(1) << 30);
    k_copy_probe<<<static_cast<int>((chunk + 255) / 256), 256, 0, s>>>(
        static_cast<const v2d*>(src) + off, static_cast<v2d*>(dst) + off, chunk);
    off += chunk;
  }
  return hipGetLastError();
}

hipError_t launch_fill64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<double><<<grid_for(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<int32_t><<<grid_for(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<float><<<grid_for(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_copy64(double* d, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_copy64<<<grid_for(n), 256, 0, s>>>(d, src, n);
  return hipGetLastError();
}
hipError_t launch_cast_scaled(float* d, const double* src, const double* scale, int64_t n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_cast_scaled<<<grid_for(n), 256, 0, s>>>(d, src, scale, n);
  return hipGetLastError();
}
hipError_t launch_axpy32(double* x, const float* d, const double* scale, int64_t n,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axpy32<<<grid_for(n), 256, 0, s>>>(x, d, scale, n);
  return hipGetLastError();
}
hipError_t launch_axpy64(double* x, const double* d, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axpy64<<<grid_for(n), 256, 0, s>>>(x, d, n);
  return hipGetLastError();
}
hipError_t launch_update_values(const Layout* Lp, const double* csr, int* bad, hipStream_t s) {
  const Layout& L = *Lp;
  k_update_slots<<<grid_for(L.epad), 256, 0, s>>>(L.epad, L.val_src, L.aT_src, csr, L.val,
                                                  L.aT);
  k_update_diag<<<nblocks(L.n), 256, 0, s>>>(L.n, L.diag_src, csr, L.diag, bad);
  return hipGetLastError();
}
hipError_t launch_gather_messages(const Layout* Lp, const double* lam, bool lam_outgoing,
                                  const double* msg, const float* msg32, double* out_lam,
                                  double* out_msg, hipStream_t s) {
  const Layout& L = *Lp;
  hipError_t e;
  if (out_lam && (e = launch_fill64(out_lam, L.nnz, 0.0, s)) != hipSuccess) return e;
  if (out_msg && (e = launch_fill64(out_msg, L.nnz, 0.0, s)) != hipSuccess) return e;
  if (L.epad <= 0) return hipSuccess;
  k_gather_messages<<<grid_for(L.epad), 256, 0, s>>>(L.epad, L.val_src, L.rev, lam,
                                                     lam_outgoing ? 1 : 0, msg, msg32, out_lam,
                                                     out_msg);
  return hipGetLastError();
}
hipError_t launch_entry_grad(const Layout* Lp, const double* lam, const double* x, double* G,
                             hipStream_t s) {
  const Layout& L = *Lp;
  if (L.nnz <= 0) return hipSuccess;
  k_entry_grad<<<grid_for(L.nnz), 256, 0, s>>>(L.nnz, L.csr_row, L.csr_col, lam, x, G);
  return hipGetLastError();
}
hipError_t launch_param_reduce(int32_t np, const int32_t* jptr, const int32_t* jnnz,
                               const double* jw, const double* lam, const double* x,
                               const int32_t* row, const int32_t* col, double* out,
                               hipStream_t s) {
  if (np <= 0) return hipSuccess;
  k_param_reduce<<<nblocks(np), 256, 0, s>>>(np, jptr, jnnz, jw, lam, x, row, col, out);
  return hipGetLastError();
}

hipError_t launch_restrict_fw(int nc, const double* rf, double* bc, hipStream_t s) {
  const int64_t m = (int64_t)nc * nc;
  k_restrict_fw<<<nblocks(m), 256, 0, s>>>(nc, rf, bc);
  return hipGetLastError();
}
hipError_t launch_prolong_add(int nc, const double* ec, double* xf, hipStream_t s) {
  const int64_t m = (int64_t)(2 * nc + 1) * (2 * nc + 1);
  k_prolong_add<<<nblocks(m), 256, 0, s>>>(nc, ec, xf);
  return hipGetLastError();
}
hipError_t launch_rbgs(const Layout* Lp, int side, int colour, const double* b, double* x,
                       hipStream_t s) {
  const Layout& L = *Lp;
  k_rbgs<0><<<nblocks(L.nlanes), kBlock, 0, s>>>(L.nlanes, side, colour, L.sptr, L.col, L.val,
                                                 L.diag, b, x, L.perm);
  return hipGetLastError();
}
hipError_t launch_dense_matvec(int n, const double* inv, const double* b, double* x,
                               hipStream_t s) {
  k_dense_matvec<<<nblocks(n), 256, 0, s>>>(n, inv, b, x);
  return hipGetLastError();
}

}  // namespace gabp
