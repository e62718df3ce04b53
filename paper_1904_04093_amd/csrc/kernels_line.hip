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

// The same index for the striped position threadIdx.x + j * kLT and for the thread's own
// position t0 + k (0 <= k < NPL): one base register plus immediate offsets.
template <int NPL>
__device__ inline int sidx(int j) {
  const int tid = threadIdx.x;
  return tid + tid / NPL + j * (kLT + kLT / NPL);
}
template <int NPL>
__device__ inline int bidx(int k) { return static_cast<int>(threadIdx.x) * (NPL + 1) + k; }

// Striped positions threadIdx.x + j * kLT of a line of len >= 1 positions. Whether stripe
// j is whole is uniform (j is a compile-time index), so the per-lane tests need no
// register per stripe. In the one partial stripe every lane still loads (its index
// clamped to the last position; the value past the end is never used): no load sits in a
// branch whose end would make the wave wait for it.
__device__ inline bool in_stripe(int j, int len) {
  return (j + 1) * kLT <= len || (j * kLT < len && static_cast<int>(threadIdx.x) < len - j * kLT);
}
template <typename T, bool NT = false>
__device__ inline T ld_stripe(const T* __restrict__ p, int j, int len) {
  const unsigned t = threadIdx.x + j * kLT;
  const unsigned i = (j + 1) * kLT <= len ? t : min(t, static_cast<unsigned>(len) - 1u);
  if constexpr (NT) return __builtin_nontemporal_load(p + i);
  else return p[i];
}

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

// Forward (from the low threads) and backward (from the high threads) scans at once, so
// the two shuffle/multiply chains overlap.
__device__ void pm_block_scan2(PM F, PM Bk, PM* totf, PM* totb, V3* vf, V3* vb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const PM Yf = pm_shfl<false>(F, off);
    const PM Yb = pm_shfl<true>(Bk, off);
    if (lane >= off) {
      F = pm_mul(F, Yf);
      pm_scale(F);
    }
    if (lane + off < 64) {
      Bk = pm_mul(Bk, Yb);
      pm_scale(Bk);
    }
  }
  if (lane == 63) totf[w] = F;
  if (lane == 0) totb[w] = Bk;
  __syncthreads();
  V3 a{1.0, 0.0, 0.0}, c{1.0, 0.0, 0.0};
  for (int q = 0; q < w; ++q) {
    a = pm_apply(totf[q], a);
    v3_scale(a);
  }
  for (int q = kLWaves - 1; q > w; --q) {
    c = pm_apply(totb[q], c);
    v3_scale(c);
  }
  PM Ef = pm_shfl<false>(F, 1);
  PM Eb = pm_shfl<true>(Bk, 1);
  if (lane == 0) Ef = pm_identity();
  if (lane == 63) Eb = pm_identity();
  *vf = pm_apply(Ef, a);
  *vb = pm_apply(Eb, c);
  __syncthreads();
}

// Affine maps g -> A g + B of the mean-only recurrences: forward and backward scans at once.
// Returns every thread's incoming g (from the low threads) and q (from the high threads).
template <typename T>
__device__ void affine_block_scan2(T Af, T Bf, T Ab, T Bb, T* tot, T* gin, T* qin) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const T Yfa = shfl<false>(Af, off), Yfb = shfl<false>(Bf, off);
    const T Yba = shfl<true>(Ab, off), Ybb = shfl<true>(Bb, off);
    if (lane >= off) {
      Bf = fma(Af, Yfb, Bf);
      Af = Af * Yfa;
    }
    if (lane + off < 64) {
      Bb = fma(Ab, Ybb, Bb);
      Ab = Ab * Yba;
    }
  }
  if (lane == 63) {
    tot[4 * w] = Af;
    tot[4 * w + 1] = Bf;
  }
  if (lane == 0) {
    tot[4 * w + 2] = Ab;
    tot[4 * w + 3] = Bb;
  }
  __syncthreads();
  T g = T(0), q = T(0);
  for (int k = 0; k < w; ++k) g = fma(tot[4 * k], g, tot[4 * k + 1]);
  for (int k = kLWaves - 1; k > w; --k) q = fma(tot[4 * k + 2], q, tot[4 * k + 3]);
  T Efa = shfl<false>(Af, 1), Efb = shfl<false>(Bf, 1);
  T Eba = shfl<true>(Ab, 1), Ebb = shfl<true>(Bb, 1);
  if (lane == 0) {
    Efa = T(1);
    Efb = T(0);
  }
  if (lane == 63) {
    Eba = T(1);
    Ebb = T(0);
  }
  *gin = fma(Efa, g, Efb);
  *qin = fma(Eba, q, Ebb);
  __syncthreads();
}

__device__ inline double wave_max64(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Striped registers (position threadIdx.x + j * kLT in slot j) into LDS.
template <int NPL, typename T>
__device__ inline void stage_regs(T* sh, const T* vals, int len) {
#pragma unroll
  for (int j = 0; j < NPL; ++j)
    if (in_stripe(j, len)) sh[sidx<NPL>(j)] = vals[j];
  __syncthreads();
}

template <int NPL, typename T>
__device__ inline void stage_take(const T* sh, int t0, int len, T pad, T* out) {
#pragma unroll
  for (int k = 0; k < NPL; ++k) out[k] = t0 + k < len ? sh[bidx<NPL>(k)] : pad;
}

// Blocked values of every thread to a line array through LDS (coalesced stores).
template <int NPL, typename T>
__device__ inline void stage_out(T* sh, const T* vals, int t0, int len) {
#pragma unroll
  for (int k = 0; k < NPL; ++k)
    if (t0 + k < len) sh[bidx<NPL>(k)] = vals[k];
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Joint line update (precision and mean messages), or with FIN the frozen-Lambda
// multipliers alpha_t = lo_t / f_{t-1}, beta_t = hi_t / h_{t+1} from the incoming
// precision messages. One block per line; blocks [0, nblk0) take side a0, the rest a1.
// ---------------------------------------------------------------------------------------
template <int NPL, bool FIN>
__global__ __launch_bounds__(kLT, 2) void k_line_joint(LineArgs a0, LineArgs a1, int nblk0) {
  __shared__ double sh[kLT * (NPL + 1)];
  __shared__ PM totf[kLWaves], totb[kLWaves];
  __shared__ double red[2][kLWaves];
  const bool second = static_cast<int>(blockIdx.x) >= nblk0;
  const LineArgs A = second ? a1 : a0;
  const int line = second ? blockIdx.x - nblk0 : blockIdx.x;
  const int len = A.len;
  const int64_t base = static_cast<int64_t>(line) * len;
  const int t0 = threadIdx.x * NPL;

  // every global load of the line is issued before the first LDS round (striped order,
  // coalesced); the LDS rounds then hand each thread its NPL consecutive positions
  double d[NPL], c[NPL], lo[NPL], h[NPL + 1];
  double lo_next;
  {
    double gd[NPL], gc[NPL], gl[NPL], gh[NPL];
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      // null incoming arrays: the other orientation's messages are zero (first update
      // after a reset)
      gd[j] = ld_stripe(A.diag + base, j, len) +
              (A.lam_in ? ld_stripe(A.lam_in + base, j, len) : 0.0);
      gc[j] = ld_stripe(A.b + base, j, len) + (A.m_in ? ld_stripe(A.m_in + base, j, len) : 0.0);
      gl[j] = ld_stripe(A.lo + base, j, len);
      gh[j] = ld_stripe(A.hi + base, j, len);
    }
    stage_regs<NPL>(sh, gd, len);
    stage_take<NPL>(sh, t0, len, 1.0, d);
    __syncthreads();
    stage_regs<NPL>(sh, gc, len);
    stage_take<NPL>(sh, t0, len, 0.0, c);
    __syncthreads();
    stage_regs<NPL>(sh, gl, len);
    stage_take<NPL>(sh, t0, len, 0.0, lo);
    lo_next = t0 + NPL < len ? sh[pidx<NPL>(t0 + NPL)] : 0.0;
    __syncthreads();
    stage_regs<NPL>(sh, gh, len);
#pragma unroll
    for (int k = 0; k < NPL; ++k) h[k + 1] = t0 + k < len ? sh[bidx<NPL>(k)] : 0.0;
    h[0] = (t0 > 0 && t0 - 1 < len) ? sh[pidx<NPL>(t0 - 1)] : 0.0;
    __syncthreads();
  }

  // per-thread maps of the forward (f_t, g_t) and backward (h_t, q_t) eliminations, and
  // every thread's incoming state from both ends of the line
  V3 vf, vb;
  {
    PM Pf = pm_identity(), Pb = pm_identity();
#pragma unroll
    for (int k = 0; k < NPL; ++k)
      if (t0 + k < len) Pf = pm_step(Pf, d[k], lo[k] * h[k], c[k], lo[k]);
#pragma unroll
    for (int k = NPL - 1; k >= 0; --k)
      if (t0 + k < len) {
        const double lnx = k + 1 < NPL ? lo[k + 1] : lo_next;
        Pb = pm_step(Pb, d[k], lnx * h[k + 1], c[k], h[k + 1]);
      }
    pm_scale(Pf);
    pm_scale(Pb);
    pm_block_scan2(Pf, Pb, totf, totb, &vf, &vb);
  }

  // forward elimination: f_t, g_t
  double Fl[NPL], Fm[NPL];
  double Sf[FIN ? NPL : 1];   // FIN: f_t + h_t - d_t, the line's Schur complement at t
  {
    double fp = vf.x / vf.y, gp = vf.z / vf.y;   // f_{t0-1}, g_{t0-1} (unused when t0 == 0)
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
      if constexpr (FIN) Sf[k] = fp;
    }
  }
  // backward elimination: h_t, q_t
  {
    double hn = vb.x / vb.y, qn = vb.z / vb.y;   // h_{t0+NPL}, q_{t0+NPL}
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
      if constexpr (FIN) {
        Fm[k] = be;
        Sf[k] += bl;
      } else {
        Fl[k] += bl;
        Fm[k] += bm;
      }
    }
  }

  if constexpr (FIN) {
    stage_out<NPL>(sh, Fl, t0, len);
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      const int t = threadIdx.x + j * kLT;
      if (t < len) {
        const double v = sh[sidx<NPL>(j)];
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
        const double v = sh[sidx<NPL>(j)];
        A.beta[base + t] = v;
        A.beta32[base + t] = static_cast<float>(v);
      }
    }
    if (A.invS) {
      __syncthreads();
      stage_out<NPL>(sh, Sf, t0, len);
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int t = threadIdx.x + j * kLT;
        if (t < len) {
          const double v = 1.0 / sh[sidx<NPL>(j)];
          A.invS[base + t] = v;
          A.invS32[base + t] = static_cast<float>(v);
        }
      }
    }
    return;
  }

  double dmax = 0.0, lmax = 0.0;
  double prev[NPL];   // the messages being replaced (Lt phase: the change per sweep)
  if (A.partials) {
#pragma unroll
    for (int j = 0; j < NPL; ++j) prev[j] = ld_stripe(A.lam_out + base, j, len);
  }
  stage_out<NPL>(sh, Fl, t0, len);
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int t = threadIdx.x + j * kLT;
    if (t < len) {
      const double v = sh[sidx<NPL>(j)];
      if (A.partials) {
        const double dv = fabs(v - prev[j]);
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
    if (t < len) A.m_out[base + t] = sh[sidx<NPL>(j)];
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
template <typename T, int NPL, bool NT>
__global__ __launch_bounds__(kLT, 3) void k_line_mean(LineMeanArgs<T> a0, LineMeanArgs<T> a1,
                                                   int nblk0) {
  __shared__ T sh[kLT * (NPL + 1)];
  __shared__ T tot[4 * kLWaves];
  const bool second = static_cast<int>(blockIdx.x) >= nblk0;
  const LineMeanArgs<T> A = second ? a1 : a0;
  const int line = second ? blockIdx.x - nblk0 : blockIdx.x;
  const int len = A.len;
  const int64_t base = static_cast<int64_t>(line) * len;
  const int t0 = threadIdx.x * NPL;

  T al[NPL], be[NPL], c[NPL], out[NPL];
  {
    T ga[NPL], gb[NPL], gc[NPL];
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      ga[j] = ld_stripe<T, NT>(A.alpha + base, j, len);
      gb[j] = ld_stripe<T, NT>(A.beta + base, j, len);
      gc[j] = ld_stripe<T, NT>(A.b + base, j, len) +
              (A.m_in ? ld_stripe<T, NT>(A.m_in + base, j, len) : T(0));
    }
    stage_regs<NPL>(sh, ga, len);
    stage_take<NPL>(sh, t0, len, T(0), al);
    __syncthreads();
    stage_regs<NPL>(sh, gb, len);
    stage_take<NPL>(sh, t0, len, T(0), be);
    __syncthreads();
    stage_regs<NPL>(sh, gc, len);
    stage_take<NPL>(sh, t0, len, T(0), c);
    __syncthreads();
  }

  T g, q;
  {
    T Af = T(1), Bf = T(0), Ab = T(1), Bb = T(0);
#pragma unroll
    for (int k = 0; k < NPL; ++k)
      if (t0 + k < len) {
        Bf = fma(-al[k], Bf, c[k]);
        Af = -al[k] * Af;
      }
#pragma unroll
    for (int k = NPL - 1; k >= 0; --k)
      if (t0 + k < len) {
        Bb = fma(-be[k], Bb, c[k]);
        Ab = -be[k] * Ab;
      }
    affine_block_scan2<T>(Af, Bf, Ab, Bb, tot, &g, &q);
  }
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    const T f = -al[k] * g;
    g = c[k] + f;
    out[k] = f;
  }
#pragma unroll
  for (int k = NPL - 1; k >= 0; --k) {
    const T bk = -be[k] * q;
    q = c[k] + bk;
    out[k] += bk;
  }
  stage_out<NPL>(sh, out, t0, len);
#pragma unroll
  for (int j = 0; j < NPL; ++j)
    if (in_stripe(j, len)) A.m_out[base + threadIdx.x + j * kLT] = sh[sidx<NPL>(j)];
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
  // null row messages: zero (first flood update after a reset)
  const double M = b[i] + (m_r ? m_r[i] : 0.0) + m_c[i];
  x[i] = invS ? M * invS[i] : M / (diag[i] + (lam_r ? lam_r[i] : 0.0) + lam_c[i]);
}

__global__ void k_line_readoff32(int64_t n, const float* __restrict__ b, const float* __restrict__ m_r,
                                 const float* __restrict__ m_c, const float* __restrict__ invS,
                                 float* __restrict__ x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  x[i] = (b[i] + (m_r ? m_r[i] : 0.0f) + m_c[i]) * invS[i];
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
  // the hint is a property of the context (both orientations of one sweep)
  if (a0.nt) {
    switch (npl) {
      case 1: k_line_mean<T, 1, true><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 2: k_line_mean<T, 2, true><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 4: k_line_mean<T, 4, true><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 8: k_line_mean<T, 8, true><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 16: k_line_mean<T, 16, true><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (npl) {
      case 1: k_line_mean<T, 1, false><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 2: k_line_mean<T, 2, false><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 4: k_line_mean<T, 4, false><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 8: k_line_mean<T, 8, false><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      case 16: k_line_mean<T, 16, false><<<nblk, kLT, 0, s>>>(a0, a1, nblk0); break;
      default: return hipErrorInvalidValue;
    }
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

hipError_t launch_gather_values(int64_t n, const int32_t* src, const double* val, double* dst,
                                hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather_values<<<elem_blocks(n), 256, 0, s>>>(n, src, val, dst);
  return hipGetLastError();
}

}  // namespace gabp
