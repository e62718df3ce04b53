// Batches of independent systems with R right-hand sides each (R = 1, 2 or 4).
//
// The batch is solved as one block-diagonal context: every flood sweep advances all
// unfinished systems at once, the precision messages Lt* (b-independent, Sec. 2.3) are
// computed once per system and shared by its right-hand sides, and each (system, rhs)
// pair keeps its own convergence state on the device, so a finished system's wavefronts
// exit at once while the others continue. The host only reads one counter per check.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gabp_batch.h"
#include "graph.h"

using namespace gabp;

namespace gabp {

void batch_free(Batch* B) {
  auto F = [](void* p) {
    if (p) (void)hipFree(p);
  };
  F(B->ext_off); F(B->int_off); F(B->slice_sys); F(B->sys_slice0); F(B->sys_on); F(B->sys_live);
  F(B->count); F(B->flags); F(B->stat); F(B->scale); F(B->best); F(B->rn); F(B->since);
  F(B->inner);
  F(B->partials); F(B->norms); F(B->b); F(B->x); F(B->r); F(B->r32); F(B->d32); F(B->dbest32);
  for (int q = 0; q < 2; ++q) {
    F(B->msg64[q]);
    F(B->msg32[q]);
  }
  if (B->host_count) (void)hipHostFree(B->host_count);
}

}  // namespace gabp

namespace {

template <typename T>
int dalloc(T** p, int64_t count) {
  GABP_HIP(hipMalloc(reinterpret_cast<void**>(p), static_cast<size_t>(std::max<int64_t>(count, 1)) * sizeof(T)));
  return GABP_OK;
}

int read_count(Batch* B, hipStream_t s, int* out) {
  GABP_HIP(hipMemcpyAsync(B->host_count, B->count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GABP_HIP(hipStreamSynchronize(s));
  *out = *B->host_count;
  return GABP_OK;
}

int finish(gabp_ctx* c, Batch* B, double* X, gabp_info* infos, int lsw, hipStream_t s) {
  GABP_HIP(batch_unpack(c, B, B->x, X, s));
  const int np = B->nsys * B->R;
  std::vector<uint32_t> flags(np);
  std::vector<PairStat> stat(np);
  GABP_HIP(hipMemcpyAsync(flags.data(), B->flags, np * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  GABP_HIP(hipMemcpyAsync(stat.data(), B->stat, np * sizeof(PairStat), hipMemcpyDeviceToHost, s));
  GABP_HIP(hipStreamSynchronize(s));
  int worst = GABP_OK;
  for (int i = 0; i < np; ++i) {
    int st = GABP_OK;
    if (flags[i] & kPairFailed) st = (stat[i].rel_res2 == stat[i].rel_res2) ? GABP_MAXSWEEPS : GABP_ENUMERIC;
    else if (!(flags[i] & kPairDone)) st = GABP_MAXSWEEPS;
    if (st == GABP_ENUMERIC) worst = GABP_ENUMERIC;
    else if (st == GABP_MAXSWEEPS && worst == GABP_OK) worst = GABP_MAXSWEEPS;
    if (infos) {
      infos[i].status = st;
      infos[i].sweeps = stat[i].sweeps;
      infos[i].lambda_sweeps = lsw;
      infos[i].outer_iters = stat[i].outer;
      infos[i].rel_res2 = stat[i].rel_res2;
      infos[i].res_inf = stat[i].res_inf;
    }
  }
  return worst;
}

int reset_pairs(gabp_ctx* c, Batch* B, hipStream_t s) {
  const int np = B->nsys * B->R;
  GABP_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(B->flags), np, 0, s));
  GABP_HIP(launch_fill_i32(B->sys_on, B->nsys, 1, s));
  GABP_HIP(launch_fill_i32(B->sys_live, B->nsys, 1, s));
  GABP_HIP(launch_fill64(reinterpret_cast<double*>(B->stat), np * (int64_t)sizeof(PairStat) / 8, 0.0, s));
  GABP_HIP(launch_fill64(B->x, static_cast<int64_t>(c->L.n) * B->R, 0.0, s));
  return GABP_OK;
}

int solve_plain(gabp_ctx* c, Batch* B, double tol, int max_sweeps, hipStream_t s) {
  const bool joint = c->opt.mode == GABP_MODE_JOINT;
  const int64_t ER = (c->L.epad + 1) * (int64_t)B->R;
  GABP_HIP(launch_fill64(B->msg64[0], ER, 0.0, s));
  if (joint) GABP_HIP(launch_fill64(c->lam[0], c->L.epad + 1, 0.0, s));
  int par = 0, done = 0, st;
  while (done < max_sweeps) {
    const int k = std::min(c->opt.check_every, max_sweeps - done);
    const int start = par;
    // one check block: k sweeps of every unfinished system, per-pair residual norms,
    // per-pair decisions, the number of systems still sweeping to the host
    st = run_block(c, *c->graphs, s, GraphKey{3, nullptr, nullptr, nullptr, start, k, 0, tol},
                   [&](hipStream_t ss) -> int {
                     int p = start;
                     for (int i = 0; i < k; ++i) {
                       double* x = i == k - 1 ? B->x : nullptr;
                       if (joint)
                         GABP_HIP(batch_joint64(c, B, c->lam[p], B->msg64[p], c->lam[p ^ 1],
                                                B->msg64[p ^ 1], x, ss));
                       else
                         GABP_HIP(batch_mean64(c, B, B->msg64[p], B->msg64[p ^ 1], x, ss));
                       p ^= 1;
                     }
                     GABP_HIP(launch_fill_i32(B->count, 1, 0, ss));
                     GABP_HIP(batch_residual(c, B, B->sys_on, B->x, nullptr, nullptr, ss));
                     GABP_HIP(batch_decide_plain(B, tol, k, ss));
                     GABP_HIP(hipMemcpyAsync(B->host_count, B->count, sizeof(int32_t),
                                             hipMemcpyDeviceToHost, ss));
                     return GABP_OK;
                   });
    if (st != GABP_OK) return st;
    par = start ^ (k & 1);
    done += k;
    GABP_HIP(hipStreamSynchronize(s));
    if (*B->host_count == 0) break;
  }
  c->parity = 0;
  return GABP_OK;
}

int solve_ir(gabp_ctx* c, Batch* B, double tol, int max_sweeps, hipStream_t s) {
  const int64_t ER = (c->L.epad + 1) * (int64_t)B->R;
  const int patience = 8;
  int total = 0, st;
  while (true) {
    GABP_HIP(launch_fill_i32(B->count, 1, 0, s));
    GABP_HIP(batch_residual(c, B, B->sys_live, B->x, nullptr, B->r, s));
    GABP_HIP(batch_ir_outer_begin(B, tol, s));
    int live = 0;
    if ((st = read_count(B, s, &live)) != GABP_OK) return st;
    if (live == 0 || total >= max_sweeps) break;
    GABP_HIP(batch_cast(c, B, s));
    GABP_HIP(batch_zero_msgs32(c, B, B->msg32[0], s));
    int par = 0, inner = 0;
    while (true) {
      const int k = std::min({c->opt.check_every, max_sweeps - total, c->opt.ir_max_inner - inner});
      const int start = par;
      // one inner block: k FP32 sweeps of the systems still inside their inner solve,
      // per-pair FP64 residuals of x + s d, best-trial tracking, count to the host
      st = run_block(c, *c->graphs, s, GraphKey{4, nullptr, nullptr, nullptr, start, k, 0, tol},
                     [&](hipStream_t ss) -> int {
                       int p = start;
                       for (int i = 0; i < k; ++i) {
                         GABP_HIP(batch_mean32(c, B, B->msg32[p], B->msg32[p ^ 1],
                                               i == k - 1 ? B->d32 : nullptr, ss));
                         p ^= 1;
                       }
                       GABP_HIP(launch_fill_i32(B->count, 1, 0, ss));
                       GABP_HIP(batch_residual(c, B, B->sys_on, B->x, B->d32, nullptr, ss));
                       GABP_HIP(batch_ir_inner_check(B, tol, c->opt.ir_inner_tol, patience, k,
                                                     c->opt.ir_max_inner, ss));
                       GABP_HIP(batch_copy_best(c, B, ss));
                       GABP_HIP(hipMemcpyAsync(B->host_count, B->count, sizeof(int32_t),
                                               hipMemcpyDeviceToHost, ss));
                       return GABP_OK;
                     });
      if (st != GABP_OK) return st;
      par = start ^ (k & 1);
      inner += k;
      total += k;
      GABP_HIP(hipStreamSynchronize(s));
      if (*B->host_count == 0 || total >= max_sweeps) break;
    }
    GABP_HIP(batch_ir_outer_end(B, s));
    GABP_HIP(batch_apply_best(c, B, s));
  }
  (void)ER;
  return GABP_OK;
}

}  // namespace

extern "C" {

int gabp_setup_batched(gabp_ctx** out, int32_t nsys, const int32_t* sys_row_off, int32_t n,
                       int64_t nnz, const int32_t* rowptr, const int32_t* col,
                       const double* val, int32_t nrhs, const gabp_options* opt,
                       hipStream_t stream) {
  if (!out || !sys_row_off || !rowptr || !col || !val) return fail(GABP_EINVAL, "NULL argument");
  *out = nullptr;
  if (nsys < 1) return fail(GABP_EINVAL, "nsys must be >= 1");
  if (nrhs != 1 && nrhs != 2 && nrhs != 4) return fail(GABP_EINVAL, "nrhs must be 1, 2 or 4");
  if (opt && (opt->schedule == GABP_SCHED_LINES || opt->schedule == GABP_SCHED_LINES_ALT))
    return fail(GABP_ENOTSUPP, "batched solves use point schedules only");
  if (opt && opt->mode == GABP_MODE_PRECOMP_SEQ)
    return fail(GABP_ENOTSUPP, "batched solves take the joint or the converged precomputed Lt");
  // the whole CSR first, so that the block-diagonal scan below reads only inside col
  if (const int st = validate(n, nnz, rowptr, col, val, nullptr); st != GABP_OK) return st;
  if (sys_row_off[0] != 0 || sys_row_off[nsys] != n) return fail(GABP_EINVAL, "sys_row_off must run from 0 to n");
  for (int s = 0; s < nsys; ++s)
    if (sys_row_off[s + 1] <= sys_row_off[s]) return fail(GABP_EINVAL, "empty or decreasing system");
  if (n <= 0 || nnz < n || rowptr[0] != 0 || rowptr[n] != nnz) return fail(GABP_EINVAL, "bad CSR sizes");
  // block-diagonal check and the slice-aligned internal numbering
  std::vector<int32_t> int_off(nsys + 1, 0);
  for (int s = 0; s < nsys; ++s) {
    const int32_t ns = sys_row_off[s + 1] - sys_row_off[s];
    int_off[s + 1] = int_off[s] + ((ns + kSlice - 1) / kSlice) * kSlice;
    for (int32_t i = sys_row_off[s]; i < sys_row_off[s + 1]; ++i)
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (col[e] < sys_row_off[s] || col[e] >= sys_row_off[s + 1])
          return fail(GABP_EINVAL, "entry couples two systems at row " + std::to_string(i));
  }
  const int32_t n_int = int_off[nsys];   // a multiple of 64: kernels rely on it
  const int64_t nnz_int = nnz + (n_int - n);
  std::vector<int32_t> rp(n_int + 1, 0), cc(nnz_int);
  std::vector<double> vv(nnz_int);
  int64_t q = 0;
  int32_t row = 0;
  for (int s = 0; s < nsys; ++s) {
    const int32_t shift = int_off[s] - sys_row_off[s];
    for (int32_t i = sys_row_off[s]; i < sys_row_off[s + 1]; ++i, ++row) {
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e, ++q) {
        cc[q] = col[e] + shift;
        vv[q] = val[e];
      }
      rp[row + 1] = static_cast<int32_t>(q);
    }
    for (; row < int_off[s + 1]; ++row) {   // padding rows: x = 0 from a unit diagonal
      cc[q] = row;
      vv[q] = 1.0;
      ++q;
      rp[row + 1] = static_cast<int32_t>(q);
    }
  }
  gabp_ctx* c = nullptr;
  int st = gabp_setup(&c, n_int, nnz_int, rp.data(), cc.data(), vv.data(), nullptr, nullptr, opt,
                      stream);
  if (st != GABP_OK) return st;
  if (c->L.max_width > 16) {
    gabp_destroy(c);
    return fail(GABP_ENOTSUPP, "batched solves support at most 16 neighbours per row");
  }
  Batch* B = new Batch();
  c->batch = B;
  B->nsys = nsys;
  B->R = nrhs;
  B->N = n;
  B->h_ext_off.assign(sys_row_off, sys_row_off + nsys + 1);
  B->h_int_off = int_off;
  const int32_t nsl = c->L.nslices;
  std::vector<int32_t> slice_sys(nsl), slice0(nsys + 1);
  for (int s = 0; s < nsys; ++s) {
    slice0[s] = int_off[s] / kSlice;
    for (int32_t k = int_off[s] / kSlice; k < int_off[s + 1] / kSlice; ++k) slice_sys[k] = s;
  }
  slice0[nsys] = nsl;
  const int np = nsys * nrhs;
  const int64_t nR = static_cast<int64_t>(n_int) * nrhs;
  const int64_t ER = (c->L.epad + 1) * static_cast<int64_t>(nrhs);
  auto bail = [&](int code) {
    gabp_destroy(c);
    return code;
  };
#define DA(p, cnt) if ((st = dalloc(&(p), cnt)) != GABP_OK) return bail(st)
  DA(B->ext_off, nsys + 1); DA(B->int_off, nsys + 1); DA(B->slice_sys, nsl); DA(B->sys_slice0, nsys + 1);
  DA(B->sys_on, nsys); DA(B->sys_live, nsys); DA(B->count, 1); DA(B->flags, np); DA(B->stat, np);
  DA(B->scale, np); DA(B->best, np); DA(B->rn, np); DA(B->since, np); DA(B->inner, np);
  DA(B->partials, static_cast<int64_t>(nsl) * nrhs * 3); DA(B->norms, np * 3);
  DA(B->b, nR); DA(B->x, nR); DA(B->r, nR); DA(B->r32, nR); DA(B->d32, nR); DA(B->dbest32, nR);
  for (int k = 0; k < 2; ++k) {
    DA(B->msg64[k], ER);
    DA(B->msg32[k], ER);
  }
#undef DA
  if (hipHostMalloc(reinterpret_cast<void**>(&B->host_count), sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
    return bail(fail(GABP_ENOMEM, "pinned counter"));
  auto up = [&](int32_t* d, const std::vector<int32_t>& h) {
    return hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
  };
  if (up(B->ext_off, B->h_ext_off) != hipSuccess || up(B->int_off, int_off) != hipSuccess ||
      up(B->slice_sys, slice_sys) != hipSuccess || up(B->sys_slice0, slice0) != hipSuccess)
    return bail(fail(GABP_EDEVICE, "batch metadata upload"));
  // message buffers start at zero: padding slots are read by every sweep, never written
  for (int k = 0; k < 2; ++k) {
    if (launch_fill64(B->msg64[k], ER, 0.0, stream) != hipSuccess ||
        launch_fill32(B->msg32[k], ER, 0.0f, stream) != hipSuccess)
      return bail(fail(GABP_EDEVICE, "batch buffer init"));
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(GABP_EDEVICE, "batch setup sync"));
  *out = c;
  return GABP_OK;
}

int gabp_solve_batched(gabp_ctx* c, const double* Bx, double* X, double tol, int32_t max_sweeps,
                       gabp_info* infos, hipStream_t s) {
  if (!c || !Bx || !X) return fail(GABP_EINVAL, "NULL argument");
  Batch* B = c->batch;
  if (!B) return fail(GABP_EINVAL, "context was not made by gabp_setup_batched");
  if (max_sweeps < 1 || !(tol >= 0.0)) return fail(GABP_EINVAL, "max_sweeps < 1 or tol < 0");
  int st, lsw = 0;
  const bool ir = c->opt.precision == GABP_F32_IR;
  if (ir || c->opt.mode == GABP_MODE_PRECOMP) {
    const bool had = c->pre[0].valid;
    if ((st = precompute(c, 0, s)) != GABP_OK) return st;
    lsw = had ? 0 : c->pre[0].sweeps;
  }
  GABP_HIP(batch_pack(c, B, Bx, B->b, s));
  if ((st = reset_pairs(c, B, s)) != GABP_OK) return st;
  st = ir ? solve_ir(c, B, tol, max_sweeps, s) : solve_plain(c, B, tol, max_sweeps, s);
  if (st != GABP_OK) return st;
  const int worst = finish(c, B, X, infos, lsw, s);
  if (worst == GABP_ENUMERIC) return fail(GABP_ENUMERIC, "a system produced non-finite values");
  return worst;
}

}  // extern "C"
