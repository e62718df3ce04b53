// HIP kernels of line GaBP: the two-sided tridiagonal line update (joint precision + mean
// messages, or mean-only with frozen precision messages), the transposes between the row
// and column layouts, and the read-off. The recurrences and layouts are described in
// gabp_line.h.
#include "gabp_line.h"

namespace gabp {
namespace {

constexpr int kLT = kLineThreads;
constexpr int kLWaves = kLT / 64;

// padded LDS index of line position t when each thread owns NPL consecutive positions:
// one pad slot per thread run keeps a thread's run start on a different bank than its
// neighbour's
template <int NPL>
__device__ inline int pidx(int t) { return t + t / NPL; }

// ---- 3x3 projective maps with the sparsity [[a b 0] [c d 0] [e f g]] -------------------
struct PM {
  double a, b, c, d, e, f, g;
};
struct V3 {
  double x, y, z;
};

__device__ inline PM pm_identity() { return PM{1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0}; }

// X * Y: apply Y first
__device__ inline PM pm_mul(const PM& X, const PM& Y) {
  PM Z;
  Z.a = fma(X.a, Y.a, X.b * Y.c);
  Z.b = fma(X.a, Y.b, X.b * Y.d);
  Z.c = fma(X.c, Y.a, X.d * Y.c);
  Z.d = fma(X.c, Y.b, X.d * Y.d);
  Z.e = fma(X.e, Y.a, fma(X.f, Y.c, X.g * Y.e));
  Z.f = fma(X.e, Y.b, fma(X.f, Y.d, X.g * Y.f));
  Z.g = X.g * Y.g;
  return Z;
}

// M_t * P with M_t = [[d, -p, 0], [1, 0, 0], [c, 0, -a]]: one step of
// (theta_t, theta_{t-1}, G_t) = M_t (theta_{t-1}, theta_{t-2}, G_{t-1})
__device__ inline PM pm_step(const PM& P, double d, double p, double c, double a) {
  PM Z;
  Z.a = fma(d, P.a, -p * P.c);
  Z.b = fma(d, P.b, -p * P.d);
  Z.c = P.a;
  Z.d = P.b;
  Z.e = fma(c, P.a, -a * P.e);
  Z.f = fma(c, P.b, -a * P.f);
  Z.g = -a * P.g;
  return Z;
}

// exact power-of-two rescaling (the maps act projectively: only ratios are used)
__device__ inline void pm_scale(PM& P) {
  const double m = fmax(fmax(fmax(fabs(P.a), fabs(P.b)), fmax(fabs(P.c), fabs(P.d))),
                        fmax(fmax(fabs(P.e), fabs(P.f)), fabs(P.g)));
  if (m > 0.0 && m <= 1.7976931348623157e308) {
    const int k = ilogb(m);
    P.a = ldexp(P.a, -k);
    P.b = ldexp(P.b, -k);
    P.c = ldexp(P.c, -k);
    P.d = ldexp(P.d, -k);
    P.e = ldexp(P.e, -k);
    P.f = ldexp(P.f, -k);
    P.g = ldexp(P.g, -k);
  }
}

__device__ inline V3 pm_apply(const PM& P, const V3& v) {
  return V3{fma(P.a, v.x, P.b * v.y), fma(P.c, v.x, P.d * v.y),
            fma(P.e, v.x, fma(P.f, v.y, P.g * v.z))};
}

__device__ inline void v3_scale(V3& v) {
  const double m = fmax(fmax(fabs(v.x), fabs(v.y)), fabs(v.z));
  if (m > 0.0 && m <= 1.7976931348623157e308) {
    const int k = ilogb(m);
    v.x = ldexp(v.x, -k);
    v.y = ldexp(v.y, -k);
    v.z = ldexp(v.z, -k);
  }
}

template <bool DOWN>
__device__ inline double shfl(double v, int off) {
  return DOWN ? __shfl_down(v, off, 64) : __shfl_up(v, off, 64);
}
template <bool DOWN>
__device__ inline float shfl(float v, int off) {
  return DOWN ? __shfl_down(v, off, 64) : __shfl_up(v, off, 64);
}

template <bool DOWN>
__device__ inline PM pm_shfl(const PM& P, int off) {
  return PM{shfl<DOWN>(P.a, off), shfl<DOWN>(P.b, off), shfl<DOWN>(P.c, off),
            shfl<DOWN>(P.d, off), shfl<DOWN>(P.e, off), shfl<DOWN>(P.f, off),
            shfl<DOWN>(P.g, off)};
}

// Incoming state of every thread from the per-thread maps P (thread order = processing
// order, reversed for REV): the start vector (1, 0, 0) pushed through the maps of all
// threads before this one. `tot` is LDS for one map per wave.
template <bool REV>
__device__ V3 pm_block_scan(PM P, PM* tot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const PM Y = pm_shfl<REV>(P, off);
    if (REV ? (lane + off < 64) : (lane >= off)) {
      P = pm_mul(P, Y);
      pm_scale(P);
    }
  }
  if (lane == (REV ? 0 : 63)) tot[w] = P;
  __syncthreads();
  V3 v{1.0, 0.0, 0.0};
  if (!REV) {
    for (int q = 0; q < w; ++q) {
      v = pm_apply(tot[q], v);
      v3_scale(v);
    }
  } else {
    for (int q = kLWaves - 1; q > w; --q) {
      v = pm_apply(tot[q], v);
      v3_scale(v);
    }
  }
  PM E = pm_shfl<REV>(P, 1);
  if (lane == (REV ? 63 : 0)) E = pm_identity();
  v = pm_apply(E, v);
  __syncthreads();
  return v;
}

// affine maps g -> A g + B, same scan for the mean-only recurrences
template <typename T, bool REV>
__device__ T affine_block_scan(T A, T B, T* totA, T* totB) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const T Ya = shfl<REV>(A, off), Yb = shfl<REV>(B, off);
    if (REV ? (lane + off < 64) : (lane >= off)) {
      B = fma(A, Yb, B);
      A = A * Ya;
    }
  }
  if (lane == (REV ? 0 : 63)) {
    totA[w] = A;
    totB[w] = B;
  }
  __syncthreads();
  T g = T(0);
  if (!REV) {
    for (int q = 0; q < w; ++q) g = fma(totA[q], g, totB[q]);
  } else {
    for (int q = kLWaves - 1; q > w; --q) g = fma(totA[q], g, totB[q]);
  }
  T Ea = shfl<REV>(A, 1), Eb = shfl<REV>(B, 1);
  if (lane == (REV ? 63 : 0)) {
    Ea = T(1);
    Eb = T(0);
  }
  g = fma(Ea, g, Eb);
  __syncthreads();
  return g;
}

__device__ inline double wave_max64(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Coalesced (striped) load of one line array (optionally plus a second one) into LDS.
template <int NPL, typename T>
__device__ inline void stage_in(T* sh, const T* __restrict__ g0, const T* __restrict__ g1,
                                int64_t base, int len) {
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int t = threadIdx.x + j * kLT;
    if (t < len) {
      T v = g0[base + t];
      if (g1) v += g1[base + t];
      sh[pidx<NPL>(t)] = v;
    }
  }
  __syncthreads();
}

template <int NPL, typename T>
__device__ inline void stage_take(const T* sh, int t0, int len, T pad, T* out) {
#pragma unroll
  for (int k = 0; k < NPL; ++k) out[k] = t0 + k < len ? sh[pidx<NPL>(t0 + k)] : pad;
}

// Blocked values of every thread to a line array through LDS (coalesced stores).
template <int NPL, typename T>
__device__ inline void stage_out(T* sh, const T* vals, int t0, int len) {
#pragma unroll
  for (int k = 0; k < NPL; ++k)
    if (t0 + k < len) sh[pidx<NPL>(t0 + k)] = vals[k];
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Joint line update (precision and mean messages), or with FIN the frozen-Lambda
// multipliers alpha_t = lo_t / f_{t-1}, beta_t = hi_t / h_{t+1} from the incoming
// precision messages. One block per line; blocks [0, nblk0) take side a0, the rest a1.
// ---------------------------------------------------------------------------------------
template <int NPL, bool FIN>
__global__ __launch_bounds__(kLT) void k_line_joint(LineArgs a0, LineArgs a1, int nblk0) {
  __shared__ double sh[kLT * (NPL + 1)];
  __shared__ PM tot[kLWaves];
  __shared__ double red[2][kLWaves];
  const bool second = static_cast<int>(blockIdx.x) >= nblk0;
  const LineArgs A = second ? a1 : a0;
  const int line = second ? blockIdx.x - nblk0 : blockIdx.x;
  const int len = A.len;
  const int64_t base = static_cast<int64_t>(line) * len;
  const int t0 = threadIdx.x * NPL;

  double d[NPL], c[NPL], lo[NPL], h[NPL + 1];
  double lo_next;
  stage_in<NPL>(sh, A.diag, A.lam_in, base, len);
  stage_take<NPL>(sh, t0, len, 1.0, d);
  __syncthreads();
  stage_in<NPL>(sh, A.b, A.m_in, base, len);
  stage_take<NPL>(sh, t0, len, 0.0, c);
  __syncthreads();
  stage_in<NPL>(sh, A.lo, static_cast<const double*>(nullptr), base, len);
  stage_take<NPL>(sh, t0, len, 0.0, lo);
  lo_next = t0 + NPL < len ? sh[pidx<NPL>(t0 + NPL)] : 0.0;
  __syncthreads();
  stage_in<NPL>(sh, A.hi, static_cast<const double*>(nullptr), base, len);
#pragma unroll
  for (int k = 0; k < NPL; ++k) h[k + 1] = t0 + k < len ? sh[pidx<NPL>(t0 + k)] : 0.0;
  h[0] = (t0 > 0 && t0 - 1 < len) ? sh[pidx<NPL>(t0 - 1)] : 0.0;
  __syncthreads();

  // forward elimination: f_t, g_t
  double Fl[NPL], Fm[NPL];
  {
    PM P = pm_identity();
#pragma unroll
    for (int k = 0; k < NPL; ++k)
      if (t0 + k < len) P = pm_step(P, d[k], lo[k] * h[k], c[k], lo[k]);
    pm_scale(P);
    const V3 v = pm_block_scan<false>(P, tot);
    double fp = v.x / v.y, gp = v.z / v.y;   // f_{t0-1}, g_{t0-1} (unused when t0 == 0)
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      const int t = t0 + k;
      double fl = 0.0, fm = 0.0, al = 0.0;
      if (t > 0 && t < len) {
        const double r = 1.0 / fp;
        fl = -lo[k] * h[k] * r;
        fm = -lo[k] * gp * r;
        al = lo[k] * r;
      }
      fp = d[k] + fl;
      gp = c[k] + fm;
      Fl[k] = FIN ? al : fl;
      Fm[k] = fm;
    }
  }
  // backward elimination: h_t, q_t
  {
    PM P = pm_identity();
#pragma unroll
    for (int k = NPL - 1; k >= 0; --k)
      if (t0 + k < len) {
        const double lnx = k + 1 < NPL ? lo[k + 1] : lo_next;
        P = pm_step(P, d[k], lnx * h[k + 1], c[k], h[k + 1]);
      }
    pm_scale(P);
    const V3 v = pm_block_scan<true>(P, tot);
    double hn = v.x / v.y, qn = v.z / v.y;   // h_{t0+NPL}, q_{t0+NPL}
#pragma unroll
    for (int k = NPL - 1; k >= 0; --k) {
      const int t = t0 + k;
      double bl = 0.0, bm = 0.0, be = 0.0;
      if (t < len - 1) {
        const double lnx = k + 1 < NPL ? lo[k + 1] : lo_next;
        const double r = 1.0 / hn;
        bl = -h[k + 1] * lnx * r;
        bm = -h[k + 1] * qn * r;
        be = h[k + 1] * r;
      }
      hn = d[k] + bl;
      qn = c[k] + bm;
      if (FIN) {
        Fm[k] = be;
      } else {
        Fl[k] += bl;
        Fm[k] += bm;
      }
    }
  }

  if (FIN) {
    stage_out<NPL>(sh, Fl, t0, len);
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      const int t = threadIdx.x + j * kLT;
      if (t < len) {
        const double v = sh[pidx<NPL>(t)];
        A.alpha[base + t] = v;
        A.alpha32[base + t] = static_cast<float>(v);
      }
    }
    __syncthreads();
    stage_out<NPL>(sh, Fm, t0, len);
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      const int t = threadIdx.x + j * kLT;
      if (t < len) {
        const double v = sh[pidx<NPL>(t)];
        A.beta[base + t] = v;
        A.beta32[base + t] = static_cast<float>(v);
      }
    }
    return;
  }

  double dmax = 0.0, lmax = 0.0;
  stage_out<NPL>(sh, Fl, t0, len);
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int t = threadIdx.x + j * kLT;
    if (t < len) {
      const double v = sh[pidx<NPL>(t)];
      if (A.partials) {
        const double dv = fabs(v - A.lam_out[base + t]);
        // a non-finite message must stop the Lt phase (fmax would drop a NaN)
        dmax = fmax(dmax, dv <= 1.7976931348623157e308 ? dv : __builtin_inf());
        lmax = fmax(lmax, fabs(v) <= 1.7976931348623157e308 ? fabs(v) : __builtin_inf());
      }
      A.lam_out[base + t] = v;
    }
  }
  __syncthreads();
  stage_out<NPL>(sh, Fm, t0, len);
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int t = threadIdx.x + j * kLT;
    if (t < len) A.m_out[base + t] = sh[pidx<NPL>(t)];
  }
  if (A.partials) {
    dmax = wave_max64(dmax);
    lmax = wave_max64(lmax);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][w] = dmax;
      red[1][w] = lmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < kLWaves; ++q) {
        dmax = fmax(dmax, red[0][q]);
        lmax = fmax(lmax, red[1][q]);
      }
      A.partials[2 * blockIdx.x] = dmax;
      A.partials[2 * blockIdx.x + 1] = lmax;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Mean-only line update with frozen precision messages (FP64 or FP32):
// g_t = c_t - alpha_t g_{t-1}, q_t = c_t - beta_t q_{t+1}, m_out = -alpha_t g_{t-1} -
// beta_t q_{t+1}, c_t = b_t + m_in(t).
// ---------------------------------------------------------------------------------------
template <typename T, int NPL>
__global__ __launch_bounds__(kLT) void k_line_mean(LineMeanArgs<T> a0, LineMeanArgs<T> a1,
                                                   int nblk0) {
  __shared__ T sh[kLT * (NPL + 1)];
  __shared__ T totA[kLWaves], totB[kLWaves];
  const bool second = static_cast<int>(blockIdx.x) >= nblk0;
  const LineMeanArgs<T> A = second ? a1 : a0;
  const int line = second ? blockIdx.x - nblk0 : blockIdx.x;
  const int len = A.len;
  const int64_t base = static_cast<int64_t>(line) * len;
  const int t0 = threadIdx.x * NPL;

  T al[NPL], be[NPL], c[NPL], out[NPL];
  stage_in<NPL>(sh, A.alpha, static_cast<const T*>(nullptr), base, len);
  stage_take<NPL>(sh, t0, len, T(0), al);
  __syncthreads();
  stage_in<NPL>(sh, A.beta, static_cast<const T*>(nullptr), base, len);
  stage_take<NPL>(sh, t0, len, T(0), be);
  __syncthreads();
  stage_in<NPL>(sh, A.b, A.m_in, base, len);
  stage_take<NPL>(sh, t0, len, T(0), c);
  __syncthreads();

  {
    T Am = T(1), Bm = T(0);
#pragma unroll
    for (int k = 0; k < NPL; ++k)
      if (t0 + k < len) {
        Bm = fma(-al[k], Bm, c[k]);
        Am = -al[k] * Am;
      }
    T g = affine_block_scan<T, false>(Am, Bm, totA, totB);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      const T f = -al[k] * g;
      g = c[k] + f;
      out[k] = f;
    }
  }
  {
    T Am = T(1), Bm = T(0);
#pragma unroll
    for (int k = NPL - 1; k >= 0; --k)
      if (t0 + k < len) {
        Bm = fma(-be[k], Bm, c[k]);
        Am = -be[k] * Am;
      }
    T q = affine_block_scan<T, true>(Am, Bm, totA, totB);
#pragma unroll
    for (int k = NPL - 1; k >= 0; --k) {
      const T bk = -be[k] * q;
      q = c[k] + bk;
      out[k] += bk;
    }
  }
  stage_out<NPL>(sh, out, t0, len);
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int t = threadIdx.x + j * kLT;
    if (t < len) A.m_out[base + t] = sh[pidx<NPL>(t)];
  }
}

// ---------------------------------------------------------------------------------------
// Tiled transpose of up to four rows x cols arrays (blockIdx.z selects the job).
// ---------------------------------------------------------------------------------------
template <typename T>
struct TJobs {
  TransposeJob<T> j[4];
};

template <typename T>
__global__ __launch_bounds__(256) void k_transpose(TJobs<T> J) {
  __shared__ T tile[32][33];
  const TransposeJob<T> jb = J.j[blockIdx.z];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  if (c0 >= jb.cols || r0 >= jb.rows) return;   // whole block
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int r = r0 + ty + k, cc = c0 + tx;
    if (r < jb.rows && cc < jb.cols) tile[ty + k][tx] = jb.src[static_cast<int64_t>(r) * jb.cols + cc];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int cc = c0 + ty + k, r = r0 + tx;
    if (cc < jb.cols && r < jb.rows) jb.dst[static_cast<int64_t>(cc) * jb.rows + r] = tile[tx][ty + k];
  }
}

// ---------------------------------------------------------------------------------------
// Read-off (row layout): x = (b + m_row + m_col) / (A_ii + Lambda_row + Lambda_col), or
// times the frozen 1/Sigma*.
// ---------------------------------------------------------------------------------------
__global__ void k_line_readoff64(int64_t n, const double* __restrict__ b,
                                 const double* __restrict__ diag, const double* __restrict__ lam_r,
                                 const double* __restrict__ m_r, const double* __restrict__ lam_c,
                                 const double* __restrict__ m_c, const double* __restrict__ invS,
                                 double* __restrict__ x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double M = b[i] + m_r[i] + m_c[i];
  x[i] = invS ? M * invS[i] : M / (diag[i] + lam_r[i] + lam_c[i]);
}

__global__ void k_line_readoff32(int64_t n, const float* __restrict__ b, const float* __restrict__ m_r,
                                 const float* __restrict__ m_c, const float* __restrict__ invS,
                                 float* __restrict__ x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  x[i] = (b[i] + m_r[i] + m_c[i]) * invS[i];
}

__global__ void k_line_invS(int64_t n, const double* __restrict__ diag, const double* __restrict__ lam_r,
                            const double* __restrict__ lam_c, double* __restrict__ invS,
                            float* __restrict__ invS32) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = 1.0 / (diag[i] + lam_r[i] + lam_c[i]);
  invS[i] = v;
  invS32[i] = static_cast<float>(v);
}

__global__ void k_gather_values(int64_t n, const int32_t* __restrict__ src,
                                const double* __restrict__ val, double* __restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t e = src[i];
  dst[i] = e >= 0 ? val[e] : 0.0;
}

inline int elem_blocks(int64_t n) { return static_cast<int>((n + 255) / 256); }

// positions per thread for lines of `len` (a power of two, at most 16)
inline int npl_for(int len) {
  int p = 1;
  while (p * kLT < len) p *= 2;
  return p;
}

template <bool FIN>
hipError_t joint_dispatch(const LineArgs& a0, const LineArgs& a1, int nblk0, int nblk, int npl,
                          hipStream_t s) {
  switch (npl) {
    case 1: k_line_joint<1, FIN><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 2: k_line_joint<2, FIN><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 4: k_line_joint<4, FIN><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 8: k_line_joint<8, FIN><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 16: k_line_joint<16, FIN><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t mean_dispatch(const LineMeanArgs<T>& a0, const LineMeanArgs<T>& a1, int nblk0,
                         int nblk, int npl, hipStream_t s) {
  switch (npl) {
    case 1: k_line_mean<T, 1><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 2: k_line_mean<T, 2><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 4: k_line_mean<T, 4><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 8: k_line_mean<T, 8><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    case 16: k_line_mean<T, 16><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t transpose_dispatch(const TransposeJob<T>* jobs, int njobs, hipStream_t s) {
  if (njobs < 1 || njobs > 4) return hipErrorInvalidValue;
  TJobs<T> J{};
  int mr = 0, mc = 0;
  for (int q = 0; q < njobs; ++q) {
    J.j[q] = jobs[q];
    mr = jobs[q].rows > mr ? jobs[q].rows : mr;
    mc = jobs[q].cols > mc ? jobs[q].cols : mc;
  }
  if (mr == 0 || mc == 0) return hipSuccess;
  const dim3 grid((mc + 31) / 32, (mr + 31) / 32, njobs);
  k_transpose<T><<<grid, 256, 0, s>>>(J);
  return hipGetLastError();
}

}  // namespace

// ---- launchers -------------------------------------------------------------------------
hipError_t launch_line_joint(const LineArgs* sides, int nsides, hipStream_t s) {
  if (nsides < 1 || nsides > 2) return hipErrorInvalidValue;
  int len = sides[0].len;
  if (nsides == 2 && sides[1].len > len) len = sides[1].len;
  if (len > kLineMaxLen) return hipErrorInvalidValue;
  const int npl = npl_for(len);
  const int nblk0 = sides[0].nlines;
  const int nblk = nblk0 + (nsides == 2 ? sides[1].nlines : 0);
  if (nblk == 0) return hipSuccess;
  const LineArgs& a1 = nsides == 2 ? sides[1] : sides[0];
  if (sides[0].alpha) return joint_dispatch<true>(sides[0], a1, nblk0, nblk, npl, s);
  return joint_dispatch<false>(sides[0], a1, nblk0, nblk, npl, s);
}

hipError_t launch_line_mean64(const LineMeanArgs<double>* sides, int nsides, hipStream_t s) {
  if (nsides < 1 || nsides > 2) return hipErrorInvalidValue;
  int len = sides[0].len;
  if (nsides == 2 && sides[1].len > len) len = sides[1].len;
  if (len > kLineMaxLen) return hipErrorInvalidValue;
  const int nblk0 = sides[0].nlines;
  const int nblk = nblk0 + (nsides == 2 ? sides[1].nlines : 0);
  if (nblk == 0) return hipSuccess;
  return mean_dispatch<double>(sides[0], nsides == 2 ? sides[1] : sides[0], nblk0, nblk,
                               npl_for(len), s);
}

hipError_t launch_line_mean32(const LineMeanArgs<float>* sides, int nsides, hipStream_t s) {
  if (nsides < 1 || nsides > 2) return hipErrorInvalidValue;
  int len = sides[0].len;
  if (nsides == 2 && sides[1].len > len) len = sides[1].len;
  if (len > kLineMaxLen) return hipErrorInvalidValue;
  const int nblk0 = sides[0].nlines;
  const int nblk = nblk0 + (nsides == 2 ? sides[1].nlines : 0);
  if (nblk == 0) return hipSuccess;
  return mean_dispatch<float>(sides[0], nsides == 2 ? sides[1] : sides[0], nblk0, nblk,
                              npl_for(len), s);
}

hipError_t launch_transpose64(const TransposeJob<double>* jobs, int njobs, hipStream_t s) {
  return transpose_dispatch<double>(jobs, njobs, s);
}

hipError_t launch_transpose32(const TransposeJob<float>* jobs, int njobs, hipStream_t s) {
  return transpose_dispatch<float>(jobs, njobs, s);
}

hipError_t launch_line_readoff64(int64_t n, const double* b, const double* diag,
                                 const double* lam_r, const double* m_r, const double* lam_c,
                                 const double* m_c, const double* invS, double* x,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_line_readoff64<<<elem_blocks(n), 256, 0, s>>>(n, b, diag, lam_r, m_r, lam_c, m_c, invS, x);
  return hipGetLastError();
}

hipError_t launch_line_readoff32(int64_t n, const float* b, const float* m_r, const float* m_c,
                                 const float* invS, float* x, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_line_readoff32<<<elem_blocks(n), 256, 0, s>>>(n, b, m_r, m_c, invS, x);
  return hipGetLastError();
}

hipError_t launch_line_invS(int64_t n, const double* diag, const double* lam_r,
                            const double* lam_c, double* invS, float* invS32, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_line_invS<<<elem_blocks(n), 256, 0, s>>>(n, diag, lam_r, lam_c, invS, invS32);
  return hipGetLastError();
}

hipError_t launch_gather_values(int64_t n, const int32_t* src, const double* val, double* dst,
                                hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather_values<<<elem_blocks(n), 256, 0, s>>>(n, src, val, dst);
  return hipGetLastError();
}

}  // namespace gabp
