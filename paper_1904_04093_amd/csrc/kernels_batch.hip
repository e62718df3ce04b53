// HIP kernels for batches of independent systems with several right-hand sides.
//
// The batch is one block-diagonal context whose systems start on slice boundaries, so
// every wavefront (slice) belongs to exactly one system: slice_sys[s] names it and a
// wavefront of a finished system exits at once. Mean messages and vectors are stored
// interleaved by right-hand side ([slot][R], [row][R]), so the R messages of a slot are
// one 4R- or 8R-byte vector load, while the precomputed Lt* and the reverse index are read
// once for all R right-hand sides (the decoupling of Sec. 2.3: Lt does not depend on b).
#include <cmath>

#include "gabp_batch.h"
#include "xcd.h"

namespace gabp {
namespace {

constexpr int kB = 256;

template <typename T, int R>
struct alignas(sizeof(T) * R) VecR {
  T v[R];
};

template <typename T, int R>
__device__ __forceinline__ VecR<T, R> ldv(const T* p) {
  return *reinterpret_cast<const VecR<T, R>*>(p);
}
template <typename T, int R>
__device__ __forceinline__ void stv(T* p, const VecR<T, R>& v) {
  *reinterpret_cast<VecR<T, R>*>(p) = v;
}

// Per-slot streams with or without non-temporal hints (NT: the sweep's footprint exceeds
// the last-level cache, so a line read or written once should not displace reused data).
template <bool NT, typename T>
__device__ __forceinline__ T ld_s(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p); else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_s(T v, T* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
}
template <bool NT, typename T, int R>
__device__ __forceinline__ VecR<T, R> ldv_s(const T* p) {
  if constexpr (NT && R > 1) {
    typedef T V __attribute__((ext_vector_type(R)));
    const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    VecR<T, R> o;
#pragma unroll
    for (int q = 0; q < R; ++q) o.v[q] = v[q];
    return o;
  } else if constexpr (NT) {
    VecR<T, R> o;
    o.v[0] = __builtin_nontemporal_load(p);
    return o;
  } else {
    return ldv<T, R>(p);
  }
}
template <bool NT, typename T, int R>
__device__ __forceinline__ void stv_s(T* p, const VecR<T, R>& o) {
  if constexpr (NT && R > 1) {
    typedef T V __attribute__((ext_vector_type(R)));
    V v;
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = o.v[q];
    __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
  } else if constexpr (NT) {
    __builtin_nontemporal_store(o.v[0], p);
  } else {
    stv<T, R>(p, o);
  }
}

// Reverse slot of p: rev[p] (int32) or p + rev16[p] (2-byte delta, when every reverse slot
// lies within int16 range of its slot, as on grids).
template <bool NT, bool R16>
__device__ __forceinline__ int rev_at(const int32_t* __restrict__ rev,
                                      const int16_t* __restrict__ rev16, int p) {
  if constexpr (R16) return p + static_cast<int>(ld_s<NT>(rev16 + p));
  else return ld_s<NT>(rev + p);
}

__device__ __forceinline__ int base_of(const int32_t* __restrict__ sptr, int j, int* w) {
  const int s = j >> 6;
  const int a = sptr[s];
  *w = (sptr[s + 1] - a) >> 6;
  return a + (j & 63);
}

// ---- mean-only sweep for R right-hand sides with a shared Lt* ---------------------------
template <typename T, int R, int KMAX, bool WX, bool NT, bool R16>
__global__ __launch_bounds__(kB) void k_mean_b(
    int n, const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const int16_t* __restrict__ rev16,
    const int32_t* __restrict__ slice_sys, const int32_t* __restrict__ sys_on,
    const uint32_t* __restrict__ pair_flags, const T* __restrict__ lamout,
    const T* __restrict__ Sx, const T* __restrict__ b, const T* msg_in, T* msg_out,
    T* __restrict__ x) {
  const int j = blockIdx.x * kB + threadIdx.x;
  if (j >= n) return;
  const int sys = slice_sys[j >> 6];
  if (!sys_on[sys]) return;
  int w;
  const int p0 = base_of(sptr, j, &w);
  VecR<T, R> M = ldv<T, R>(b + (int64_t)j * R);
  VecR<T, R> m[KMAX];
  T lo[KMAX];
  int rv[KMAX];
  // every load of the row first, the sums after: no wait between the slots' loads
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < w) {
      const int p = p0 + 64 * k;
      m[k] = ldv_s<NT, T, R>(msg_in + (int64_t)p * R);
      lo[k] = ld_s<NT>(lamout + p);
      rv[k] = rev_at<NT, R16>(rev, rev16, p);
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < w) {
#pragma unroll
      for (int q = 0; q < R; ++q) M.v[q] += m[k].v[q];
    }
  if (WX) {
    // a converged (system, rhs) pair keeps the read-off it converged with
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (!(pair_flags[sys * R + q] & kPairDone)) {
        if constexpr (sizeof(T) == 8) x[(int64_t)j * R + q] = M.v[q] / Sx[j];
        else x[(int64_t)j * R + q] = M.v[q] * Sx[j];
      }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < w) {
      VecR<T, R> o;
#pragma unroll
      for (int q = 0; q < R; ++q) o.v[q] = lo[k] * (M.v[q] - m[k].v[q]);
      stv_s<NT, T, R>(msg_out + (int64_t)rv[k] * R, o);
    }
  }
}

// ---- joint FP64 sweep for R right-hand sides (Lt updated once per slot) ---------------
template <int R, int KMAX, bool WX, bool NT, bool R16>
__global__ __launch_bounds__(kB) void k_joint_b(
    int n, const int32_t* __restrict__ sptr, const int32_t* __restrict__ rev,
    const int16_t* __restrict__ rev16,
    const int32_t* __restrict__ slice_sys, const int32_t* __restrict__ sys_on,
    const uint32_t* __restrict__ pair_flags, const double* __restrict__ coef,
    const double* __restrict__ diag, const double* __restrict__ b, const double* lam_in,
    const double* msg_in, double* lam_out, double* msg_out, double* __restrict__ x) {
  const int j = blockIdx.x * kB + threadIdx.x;
  if (j >= n) return;
  const int sys = slice_sys[j >> 6];
  if (!sys_on[sys]) return;
  int w;
  const int p0 = base_of(sptr, j, &w);
  double S = diag[j];
  VecR<double, R> M = ldv<double, R>(b + (int64_t)j * R);
  VecR<double, R> m[KMAX];
  double l[KMAX], a[KMAX];
  int rv[KMAX];
  // every load of the row first, the sums after: no wait between the slots' loads
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < w) {
      const int p = p0 + 64 * k;
      m[k] = ldv_s<NT, double, R>(msg_in + (int64_t)p * R);
      l[k] = ld_s<NT>(lam_in + p);
      a[k] = ld_s<NT>(coef + p);
      rv[k] = rev_at<NT, R16>(rev, rev16, p);
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < w) {
      S = fma(l[k], a[k], S);
#pragma unroll
      for (int q = 0; q < R; ++q) M.v[q] += m[k].v[q];
    }
  if (WX) {
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (!(pair_flags[sys * R + q] & kPairDone)) x[(int64_t)j * R + q] = M.v[q] / S;
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < w) {
      const double L = -a[k] / (S - l[k] * a[k]);
      st_s<NT>(L, lam_out + rv[k]);
      VecR<double, R> o;
#pragma unroll
      for (int q = 0; q < R; ++q) o.v[q] = L * (M.v[q] - m[k].v[q]);
      stv_s<NT, double, R>(msg_out + (int64_t)rv[k] * R, o);
    }
  }
}

// ---- residual for R right-hand sides, per-slice partial norms --------------------------
// r = b - A (x + scale * dx); partials[(slice * R + q) * 3 + {0,1,2}] = sum r^2, max|r|, sum b^2
template <int R, bool XADD>
__global__ __launch_bounds__(kB) void k_residual_b(
    int n, const int32_t* __restrict__ sptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ slice_sys, const int32_t* __restrict__ gate,
    const double* __restrict__ val, const double* __restrict__ diag,
    const double* __restrict__ b, const double* __restrict__ x, const float* __restrict__ dx,
    const double* __restrict__ scale, double* __restrict__ r, double* __restrict__ partials) {
  const int j = xcd_block(blockIdx.x, gridDim.x) * kB + threadIdx.x;
  // The internal row count n is a multiple of 64 (systems are slice-aligned), so this test
  // retires whole wavefronts: the grid rounds up to 256 threads, and the extra wavefronts
  // must not read slice_sys past its last slice.
  if (j >= n) return;
  const int slice = j >> 6;
  // every lane of a wavefront has the same slice, hence the same system
  const int sys = slice_sys[slice];
  if (!gate[sys]) return;
  double acc[R], bsq[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = bsq[q] = 0.0;
  if (j < n) {
    int w;
    const int p0 = base_of(sptr, j, &w);
    double sc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) sc[q] = XADD ? scale[sys * R + q] : 0.0;
    const VecR<double, R> bj = ldv<double, R>(b + (int64_t)j * R);
    VecR<double, R> xj = ldv<double, R>(x + (int64_t)j * R);
    if (XADD) {
#pragma unroll
      for (int q = 0; q < R; ++q) xj.v[q] = fma(sc[q], (double)dx[(int64_t)j * R + q], xj.v[q]);
    }
    const double d = diag[j];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      acc[q] = fma(-d, xj.v[q], bj.v[q]);
      bsq[q] = bj.v[q] * bj.v[q];
    }
    for (int k = 0; k < w; ++k) {
      const int p = p0 + 64 * k;
      const int c = col[p];
      const double a = val[p];
      VecR<double, R> xc = ldv<double, R>(x + (int64_t)c * R);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        double v = xc.v[q];
        if (XADD) v = fma(sc[q], (double)dx[(int64_t)c * R + q], v);
        acc[q] = fma(-a, v, acc[q]);
      }
    }
    if (r) {
      VecR<double, R> o;
#pragma unroll
      for (int q = 0; q < R; ++q) o.v[q] = acc[q];
      stv<double, R>(r + (int64_t)j * R, o);
    }
  }
  // wavefront reduction outside any divergent branch (one slice = one wavefront)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    double s2 = acc[q] * acc[q], mx = fabs(acc[q]), b2 = bsq[q];
    if (mx != mx) mx = INFINITY;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s2 += __shfl_xor(s2, o, 64);
      mx = fmax(mx, __shfl_xor(mx, o, 64));
      b2 += __shfl_xor(b2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      partials[((int64_t)slice * R + q) * 3 + 0] = s2;
      partials[((int64_t)slice * R + q) * 3 + 1] = mx;
      partials[((int64_t)slice * R + q) * 3 + 2] = b2;
    }
  }
}

// one block per system: reduce its slices' partials in slice order
template <int R>
__global__ __launch_bounds__(256) void k_sys_reduce(const int32_t* __restrict__ sys_slice0,
                                                   const int32_t* __restrict__ gate,
                                                   const double* __restrict__ partials,
                                                   double* __restrict__ norms) {
  __shared__ double sh[R][3][4];
  const int sys = blockIdx.x;
  if (!gate[sys]) return;
  const int s0 = sys_slice0[sys], s1 = sys_slice0[sys + 1];
  double a[R][3];
#pragma unroll
  for (int q = 0; q < R; ++q) a[q][0] = a[q][1] = a[q][2] = 0.0;
  for (int s = s0 + (int)threadIdx.x; s < s1; s += 256) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const double* p = partials + ((int64_t)s * R + q) * 3;
      a[q][0] += p[0];
      a[q][1] = fmax(a[q][1], p[1]);
      a[q][2] += p[2];
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a[q][0] += __shfl_xor(a[q][0], o, 64);
      a[q][1] = fmax(a[q][1], __shfl_xor(a[q][1], o, 64));
      a[q][2] += __shfl_xor(a[q][2], o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      sh[q][0][threadIdx.x >> 6] = a[q][0];
      sh[q][1][threadIdx.x >> 6] = a[q][1];
      sh[q][2][threadIdx.x >> 6] = a[q][2];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double t0 = sh[q][0][0], t1 = sh[q][1][0], t2 = sh[q][2][0];
      for (int wv = 1; wv < 4; ++wv) {
        t0 += sh[q][0][wv];
        t1 = fmax(t1, sh[q][1][wv]);
        t2 += sh[q][2][wv];
      }
      norms[(sys * R + q) * 3 + 0] = t0;
      norms[(sys * R + q) * 3 + 1] = t1;
      norms[(sys * R + q) * 3 + 2] = t2;
    }
  }
}

// ---- per-(system, rhs) decisions: one thread per system ------------------------------
__device__ __forceinline__ double rel_of(const double* nm) {
  const double bn = sqrt(nm[2]);
  return bn > 0 ? sqrt(nm[0]) / bn : sqrt(nm[0]);
}

// plain solves: a pair is done once its relative residual reaches tol
__global__ void k_decide_plain(int nsys, int R, double tol, int k_swept,
                               const double* __restrict__ norms, uint32_t* __restrict__ flags,
                               PairStat* __restrict__ stat, int32_t* __restrict__ sys_on,
                               int32_t* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || !sys_on[s]) return;
  int live = 0;
  for (int q = 0; q < R; ++q) {
    const int i = s * R + q;
    if (flags[i] & kPairDone) continue;
    const double* nm = norms + i * 3;
    const double rel = rel_of(nm);
    stat[i].rel_res2 = rel;
    stat[i].res_inf = nm[1];
    stat[i].sweeps += k_swept;
    if (!(rel == rel) || !isfinite(nm[1])) {
      flags[i] |= kPairDone | kPairFailed;
    } else if (rel <= tol) {
      flags[i] |= kPairDone;
    } else {
      ++live;
    }
  }
  sys_on[s] = live > 0;
  if (live) atomicAdd(count, 1);
}

// refinement, start of an outer step: norms of r = b - A x decide convergence; the scale of
// the inner right-hand side is ||r||_inf
__global__ void k_ir_outer_begin(int nsys, int R, double tol, const double* __restrict__ norms,
                                 uint32_t* __restrict__ flags, PairStat* __restrict__ stat,
                                 double* __restrict__ scale, double* __restrict__ best,
                                 double* __restrict__ rn, int32_t* __restrict__ since,
                                 int32_t* __restrict__ inner,
                                 int32_t* __restrict__ sys_live, int32_t* __restrict__ sys_on,
                                 int32_t* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || !sys_live[s]) return;
  int live = 0;
  for (int q = 0; q < R; ++q) {
    const int i = s * R + q;
    if (flags[i] & kPairDone) continue;
    const double* nm = norms + i * 3;
    const double rel = rel_of(nm);
    stat[i].rel_res2 = rel;
    stat[i].res_inf = nm[1];
    if (!(rel == rel) || !isfinite(nm[1])) {
      flags[i] |= kPairDone | kPairFailed;
      continue;
    }
    if (rel <= tol || nm[0] == 0.0) {
      flags[i] |= kPairDone;
      continue;
    }
    scale[i] = nm[1];
    rn[i] = sqrt(nm[0]);
    best[i] = rn[i];
    since[i] = 0;
    inner[i] = 0;
    flags[i] &= ~(kPairHasBest | kPairInnerDone | kPairNewBest);
    ++live;
  }
  sys_live[s] = live > 0;
  sys_on[s] = live > 0;
  if (live) atomicAdd(count, 1);
}

// refinement, inner check: track the best trial correction per pair; a system keeps
// sweeping while one of its pairs is still inside its inner solve
__global__ void k_ir_inner_check(int nsys, int R, double tol, double inner_tol, int patience,
                                 int k_swept, int inner_max, const double* __restrict__ norms,
                                 uint32_t* __restrict__ flags, PairStat* __restrict__ stat,
                                 double* __restrict__ best, const double* __restrict__ rn,
                                 int32_t* __restrict__ since, int32_t* __restrict__ inner,
                                 int32_t* __restrict__ sys_on, int32_t* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || !sys_on[s]) return;
  int live = 0;
  for (int q = 0; q < R; ++q) {
    const int i = s * R + q;
    flags[i] &= ~kPairNewBest;
    if (flags[i] & kPairDone) continue;
    // every pair of a sweeping system was swept k_swept more times
    stat[i].sweeps += k_swept;
    inner[i] += k_swept;
    if (flags[i] & kPairInnerDone) continue;
    const double* nm = norms + i * 3;
    const double nt = sqrt(nm[0]);
    const double bn = sqrt(nm[2]);
    if (!(nt == nt)) {
      flags[i] |= kPairDone | kPairFailed;
      continue;
    }
    if (nt < best[i]) {
      best[i] = nt;
      flags[i] |= kPairHasBest | kPairNewBest;
      since[i] = 0;
    } else {
      since[i] += 1;
    }
    const bool done = best[i] <= inner_tol * rn[i] || (bn > 0 ? best[i] / bn : best[i]) <= tol ||
                      ((flags[i] & kPairHasBest) && since[i] >= patience) || inner[i] >= inner_max;
    if (done) flags[i] |= kPairInnerDone;
    else ++live;
  }
  sys_on[s] = live > 0;
  if (live) atomicAdd(count, 1);
}

// refinement, end of an outer step: pairs without any improving trial stagnated
__global__ void k_ir_outer_end(int nsys, int R, uint32_t* __restrict__ flags,
                               PairStat* __restrict__ stat, int32_t* __restrict__ sys_live) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || !sys_live[s]) return;
  for (int q = 0; q < R; ++q) {
    const int i = s * R + q;
    if (flags[i] & kPairDone) continue;
    stat[i].outer += 1;
    if (!(flags[i] & kPairHasBest)) flags[i] |= kPairDone | kPairFailed;
  }
}

// ---- row helpers ----------------------------------------------------------------------
template <int R>
__global__ void k_copy_best(int n, const int32_t* __restrict__ slice_sys,
                            const uint32_t* __restrict__ flags, const float* __restrict__ d,
                            float* __restrict__ dbest) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int sys = slice_sys[j >> 6];
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (flags[sys * R + q] & kPairNewBest) dbest[(int64_t)j * R + q] = d[(int64_t)j * R + q];
}

template <int R>
__global__ void k_apply_best(int n, const int32_t* __restrict__ slice_sys,
                             const uint32_t* __restrict__ flags, const double* __restrict__ scale,
                             const float* __restrict__ dbest, double* __restrict__ x) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int sys = slice_sys[j >> 6];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const uint32_t f = flags[sys * R + q];
    if ((f & kPairHasBest) && !(f & kPairDone))
      x[(int64_t)j * R + q] = fma(scale[sys * R + q], (double)dbest[(int64_t)j * R + q],
                                  x[(int64_t)j * R + q]);
  }
}

template <int R>
__global__ void k_cast_pairs(int n, const int32_t* __restrict__ slice_sys,
                             const int32_t* __restrict__ sys_on, const double* __restrict__ scale,
                             const double* __restrict__ r, float* __restrict__ r32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int sys = slice_sys[j >> 6];
  if (!sys_on[sys]) return;
#pragma unroll
  for (int q = 0; q < R; ++q)
    r32[(int64_t)j * R + q] = (float)(r[(int64_t)j * R + q] / scale[sys * R + q]);
}

// zero the mean messages a row receives (all its slots, all right-hand sides)
template <typename T, int R>
__global__ void k_zero_slots(int n, const int32_t* __restrict__ sptr,
                             const int32_t* __restrict__ slice_sys,
                             const int32_t* __restrict__ sys_on, T* __restrict__ msg) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (sys_on && !sys_on[slice_sys[j >> 6]]) return;
  int w;
  const int p0 = base_of(sptr, j, &w);
  for (int k = 0; k < w; ++k)
#pragma unroll
    for (int q = 0; q < R; ++q) msg[(int64_t)(p0 + 64 * k) * R + q] = T(0);
}

// external [R][N] <-> internal [n_int][R]
template <int R>
__global__ void k_pack(int n_int, const int32_t* __restrict__ slice_sys,
                       const int32_t* __restrict__ int_off, const int32_t* __restrict__ ext_off,
                       int64_t N, const double* __restrict__ Bx, double* __restrict__ bi) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_int) return;
  const int s = slice_sys[j >> 6];
  const int local = j - int_off[s];
  const bool real = local < ext_off[s + 1] - ext_off[s];
#pragma unroll
  for (int q = 0; q < R; ++q)
    bi[(int64_t)j * R + q] = real ? Bx[q * N + ext_off[s] + local] : 0.0;
}
template <int R>
__global__ void k_unpack(int n_int, const int32_t* __restrict__ slice_sys,
                         const int32_t* __restrict__ int_off, const int32_t* __restrict__ ext_off,
                         int64_t N, const double* __restrict__ xi, double* __restrict__ X) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_int) return;
  const int s = slice_sys[j >> 6];
  const int local = j - int_off[s];
  if (local >= ext_off[s + 1] - ext_off[s]) return;
#pragma unroll
  for (int q = 0; q < R; ++q) X[q * N + ext_off[s] + local] = xi[(int64_t)j * R + q];
}

inline int nb(int64_t n, int b = kB) { return static_cast<int>((n + b - 1) / b); }

// Whether a batched sweep streams its per-slot arrays with non-temporal hints: its bytes
// per sweep (per slot and per row, for R right-hand sides) against the 256 MiB last-level
// cache, with the single-system sweeps' thresholds (1x for FP64, 2x for FP32).
inline bool stream_hints(const Layout& L, double per_slot, double per_row, double factor) {
  constexpr double kLLC = 256.0 * 1024 * 1024;
  return per_slot * static_cast<double>(L.epad) + per_row * static_cast<double>(L.n) >
         factor * kLLC;
}

}  // namespace

// ---------------------------------------------------------------------------------------
#define GABP_R_DISPATCH(R, ...)                          \
  switch (R) {                                           \
    case 1: { constexpr int RR = 1; __VA_ARGS__; break; } \
    case 2: { constexpr int RR = 2; __VA_ARGS__; break; } \
    case 4: { constexpr int RR = 4; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;                \
  }

#define GABP_B_NT_DISPATCH(NTV, ...)                 \
  if (NTV) { constexpr bool NN = true; __VA_ARGS__; }   \
  else { constexpr bool NN = false; __VA_ARGS__; }

#define GABP_B_R16_DISPATCH(R16V, ...)                 \
  if (R16V) { constexpr bool RV = true; __VA_ARGS__; }   \
  else { constexpr bool RV = false; __VA_ARGS__; }

#define GABP_K_DISPATCH(W, ...)                                 \
  if ((W) <= 4) { constexpr int KK = 4; __VA_ARGS__; }          \
  else if ((W) <= 8) { constexpr int KK = 8; __VA_ARGS__; }     \
  else if ((W) <= 16) { constexpr int KK = 16; __VA_ARGS__; }   \
  else { return hipErrorInvalidValue; }

hipError_t batch_mean32(const gabp_ctx* c, const Batch* B, const float* msg_in, float* msg_out,
                        float* x, hipStream_t s) {
  const Layout& L = c->L;
  const Precomp& P = c->pre[0];
  const int g = nb(L.n);
  const bool nt = stream_hints(L, 8.0 + 8.0 * B->R, 4.0 * B->R, 2.0);
  GABP_R_DISPATCH(B->R, GABP_K_DISPATCH(L.max_width, GABP_B_NT_DISPATCH(nt, GABP_B_R16_DISPATCH(L.rev16 != nullptr && !L.rev16_classed, {
    if (x) k_mean_b<float, RR, KK, true, NN, RV><<<g, kB, 0, s>>>(L.n, L.sptr, L.rev, L.rev16, B->slice_sys, B->sys_on, B->flags, P.lamout32, P.invS32, B->r32, msg_in, msg_out, x);
    else k_mean_b<float, RR, KK, false, NN, RV><<<g, kB, 0, s>>>(L.n, L.sptr, L.rev, L.rev16, B->slice_sys, B->sys_on, B->flags, P.lamout32, P.invS32, B->r32, msg_in, msg_out, x);
  }))));
  return hipGetLastError();
}

hipError_t batch_mean64(const gabp_ctx* c, const Batch* B, const double* msg_in,
                        double* msg_out, double* x, hipStream_t s) {
  const Layout& L = c->L;
  const Precomp& P = c->pre[0];
  const int g = nb(L.n);
  const bool nt = stream_hints(L, 12.0 + 16.0 * B->R, 8.0 * B->R, 1.0);
  GABP_R_DISPATCH(B->R, GABP_K_DISPATCH(L.max_width, GABP_B_NT_DISPATCH(nt, GABP_B_R16_DISPATCH(L.rev16 != nullptr && !L.rev16_classed, {
    if (x) k_mean_b<double, RR, KK, true, NN, RV><<<g, kB, 0, s>>>(L.n, L.sptr, L.rev, L.rev16, B->slice_sys, B->sys_on, B->flags, P.lamout, P.S, B->b, msg_in, msg_out, x);
    else k_mean_b<double, RR, KK, false, NN, RV><<<g, kB, 0, s>>>(L.n, L.sptr, L.rev, L.rev16, B->slice_sys, B->sys_on, B->flags, P.lamout, P.S, B->b, msg_in, msg_out, x);
  }))));
  return hipGetLastError();
}

hipError_t batch_joint64(const gabp_ctx* c, const Batch* B, const double* lam_in,
                         const double* msg_in, double* lam_out, double* msg_out, double* x,
                         hipStream_t s) {
  const Layout& L = c->L;
  const int g = nb(L.n);
  const bool nt = stream_hints(L, 28.0 + 16.0 * B->R, 8.0 + 8.0 * B->R, 1.0);
  GABP_R_DISPATCH(B->R, GABP_K_DISPATCH(L.max_width, GABP_B_NT_DISPATCH(nt, GABP_B_R16_DISPATCH(L.rev16 != nullptr && !L.rev16_classed, {
    if (x) k_joint_b<RR, KK, true, NN, RV><<<g, kB, 0, s>>>(L.n, L.sptr, L.rev, L.rev16, B->slice_sys, B->sys_on, B->flags, L.aT, L.diag, B->b, lam_in, msg_in, lam_out, msg_out, x);
    else k_joint_b<RR, KK, false, NN, RV><<<g, kB, 0, s>>>(L.n, L.sptr, L.rev, L.rev16, B->slice_sys, B->sys_on, B->flags, L.aT, L.diag, B->b, lam_in, msg_in, lam_out, msg_out, x);
  }))));
  return hipGetLastError();
}

hipError_t batch_residual(const gabp_ctx* c, const Batch* B, const int32_t* gate,
                          const double* x, const float* dx, double* r, hipStream_t s) {
  const Layout& L = c->L;
  const int g = nb(static_cast<int64_t>(L.nslices) * 64);
  GABP_R_DISPATCH(B->R, {
    if (dx) k_residual_b<RR, true><<<g, kB, 0, s>>>(L.n, L.sptr, L.col, B->slice_sys, gate, L.val, L.diag, B->b, x, dx, B->scale, r, B->partials);
    else k_residual_b<RR, false><<<g, kB, 0, s>>>(L.n, L.sptr, L.col, B->slice_sys, gate, L.val, L.diag, B->b, x, nullptr, nullptr, r, B->partials);
    k_sys_reduce<RR><<<B->nsys, 256, 0, s>>>(B->sys_slice0, gate, B->partials, B->norms);
  });
  return hipGetLastError();
}

hipError_t batch_decide_plain(const Batch* B, double tol, int k_swept, hipStream_t s) {
  k_decide_plain<<<nb(B->nsys), kB, 0, s>>>(B->nsys, B->R, tol, k_swept, B->norms, B->flags,
                                            B->stat, B->sys_on, B->count);
  return hipGetLastError();
}

hipError_t batch_ir_outer_begin(const Batch* B, double tol, hipStream_t s) {
  k_ir_outer_begin<<<nb(B->nsys), kB, 0, s>>>(B->nsys, B->R, tol, B->norms, B->flags, B->stat,
                                              B->scale, B->best, B->rn, B->since, B->inner,
                                              B->sys_live, B->sys_on, B->count);
  return hipGetLastError();
}

hipError_t batch_ir_inner_check(const Batch* B, double tol, double inner_tol, int patience,
                                int k_swept, int inner_max, hipStream_t s) {
  k_ir_inner_check<<<nb(B->nsys), kB, 0, s>>>(B->nsys, B->R, tol, inner_tol, patience,
                                              k_swept, inner_max, B->norms, B->flags,
                                              B->stat, B->best, B->rn, B->since, B->inner,
                                              B->sys_on, B->count);
  return hipGetLastError();
}

hipError_t batch_ir_outer_end(const Batch* B, hipStream_t s) {
  k_ir_outer_end<<<nb(B->nsys), kB, 0, s>>>(B->nsys, B->R, B->flags, B->stat, B->sys_live);
  return hipGetLastError();
}

hipError_t batch_copy_best(const gabp_ctx* c, const Batch* B, hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_copy_best<RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, B->slice_sys, B->flags, B->d32, B->dbest32)));
  return hipGetLastError();
}

hipError_t batch_apply_best(const gabp_ctx* c, const Batch* B, hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_apply_best<RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, B->slice_sys, B->flags, B->scale, B->dbest32, B->x)));
  return hipGetLastError();
}

hipError_t batch_cast(const gabp_ctx* c, const Batch* B, hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_cast_pairs<RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, B->slice_sys, B->sys_on, B->scale, B->r, B->r32)));
  return hipGetLastError();
}

hipError_t batch_zero_msgs32(const gabp_ctx* c, const Batch* B, float* msg, hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_zero_slots<float, RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, c->L.sptr, B->slice_sys, B->sys_on, msg)));
  return hipGetLastError();
}

hipError_t batch_zero_msgs64(const gabp_ctx* c, const Batch* B, double* msg, hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_zero_slots<double, RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, c->L.sptr, B->slice_sys, nullptr, msg)));
  return hipGetLastError();
}

hipError_t batch_pack(const gabp_ctx* c, const Batch* B, const double* Bx, double* bi,
                      hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_pack<RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, B->slice_sys, B->int_off, B->ext_off, B->N, Bx, bi)));
  return hipGetLastError();
}

hipError_t batch_unpack(const gabp_ctx* c, const Batch* B, const double* xi, double* X,
                        hipStream_t s) {
  GABP_R_DISPATCH(B->R, (k_unpack<RR><<<nb(c->L.n), kB, 0, s>>>(c->L.n, B->slice_sys, B->int_off, B->ext_off, B->N, xi, X)));
  return hipGetLastError();
}

}  // namespace gabp
