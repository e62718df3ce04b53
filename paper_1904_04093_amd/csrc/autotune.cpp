// Autotuner: per context, measure and pick (1) whether the sweep kernels stream their
// per-slot arrays with non-temporal hints (for tiled layouts also: non-temporal stores with
// plain loads), (2) the workgroup size of the single-system
// sweep kernels (64, 128 or 256 threads: 1, 2 or 4 slices of 64 rows) and (3) the number of
// sweeps between residual checks. Results are cached per (device, sizes, mode) in a JSON-lines file named by the
// environment variable GABP_AUTOTUNE_CACHE (in memory only when it is unset).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "gabp_batch.h"
#include "gabp_line.h"
#include "graph.h"

using namespace gabp;

namespace {

struct Tuned {
  int hints;
  int check_every;
  int block;
};

std::mutex g_mu;
std::map<std::string, Tuned> g_mem;

std::string key_of(const gabp_ctx* c) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev = prop.gcnArchName;
  char buf[256];
  // the layout hash separates layouts of one matrix (tiled or not, colour-major, lines)
  std::snprintf(buf, sizeof(buf),
                "%s|n=%d|slots=%lld|w=%d|R=%d|sys=%d|mode=%d|prec=%d|sched=%d|layout=%016llx",
                dev.c_str(), c->L.n, static_cast<long long>(c->L.epad), c->L.max_width,
                c->batch ? c->batch->R : 1, c->batch ? c->batch->nsys : 1, c->opt.mode,
                c->opt.precision, c->opt.schedule, static_cast<unsigned long long>(c->L.hash));
  return buf;
}

bool cache_lookup(const std::string& key, Tuned* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_mem.find(key);
  if (it != g_mem.end()) {
    *t = it->second;
    return true;
  }
  const char* path = std::getenv("GABP_AUTOTUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    // {"key": "...", "stream_hints": H, "check_every": C, "block": B}
    const char* k0 = std::strstr(line, "\"key\": \"");
    if (!k0) continue;
    k0 += 8;
    const char* k1 = std::strchr(k0, '"');
    if (!k1 || std::string(k0, k1) != key) continue;
    int h = 0, ce = 0;
    const char* hp = std::strstr(k1, "\"stream_hints\": ");
    const char* cp = std::strstr(k1, "\"check_every\": ");
    if (!hp || !cp) continue;
    h = std::atoi(hp + 16);
    ce = std::atoi(cp + 15);
    const char* bp = std::strstr(k1, "\"block\": ");
    const int blk = bp ? std::atoi(bp + 9) : kBlock;
    if (ce >= 1 && (blk == 64 || blk == 128 || blk == 256)) {
      *t = Tuned{h, ce, blk};
      found = true;
    }
  }
  std::fclose(f);
  if (found) g_mem[key] = *t;
  return found;
}

void cache_store(const std::string& key, const Tuned& t) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_mem[key] = t;
  const char* path = std::getenv("GABP_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"stream_hints\": %d, \"check_every\": %d, \"block\": %d}\n",
               key.c_str(), t.hints, t.check_every, t.block);
  std::fclose(f);
}

// time `reps` calls of fn(stream) on stream s, in seconds per call
template <class F>
int time_it(hipStream_t s, int reps, F&& fn, double* out) {
  hipEvent_t a, b;
  GABP_HIP(hipEventCreate(&a));
  GABP_HIP(hipEventCreate(&b));
  int st = GABP_OK;
  for (int i = 0; i < 2 && st == GABP_OK; ++i) st = fn();   // warm-up
  if (st == GABP_OK) {
    GABP_HIP(hipEventRecord(a, s));
    for (int i = 0; i < reps && st == GABP_OK; ++i) st = fn();
    GABP_HIP(hipEventRecord(b, s));
    GABP_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    GABP_HIP(hipEventElapsedTime(&ms, a, b));
    *out = ms * 1e-3 / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

// Line schedules have no stream-hint variants: only the check interval is tuned, from the
// time of one line sweep and of one residual check on a zero right-hand side.
int autotune_lines(gabp_ctx* c, int32_t* check_every_out, int32_t* hints_out, hipStream_t s) {
  const std::string key = key_of(c);
  Tuned t{};
  if (!cache_lookup(key, &t)) {
    int st;
    const bool f32 = c->opt.precision == GABP_F32_IR;
    if ((f32 || c->opt.mode == GABP_MODE_PRECOMP) && (st = precompute(c, 0, s)) != GABP_OK)
      return st;
    const int64_t n = c->L.n;
    GABP_HIP(launch_fill64(c->r, n, 0.0, s));
    if (f32) {
      if ((st = line_ensure32(c, s)) != GABP_OK) return st;
      GABP_HIP(launch_fill32(c->r32, n, 0.0f, s));
      if ((st = line_rhs32(c, c->r32, s)) != GABP_OK) return st;
      if ((st = line_reset32(c, s)) != GABP_OK) return st;
    } else {
      if ((st = line_rhs64(c, c->r, s)) != GABP_OK) return st;
      if ((st = line_reset64(c, s)) != GABP_OK) return st;
    }
    auto one_sweep = [&]() -> int {
      return f32 ? line_sweep32(c, 0, c->r32, nullptr, s) : line_sweep64(c, 0, c->r, nullptr, s);
    };
    double t_sweep = 0.0, t_check = 0.0;
    if ((st = time_it(s, 10, one_sweep, &t_sweep)) != GABP_OK) return st;
    auto one_check = [&]() -> int {
      GABP_HIP(launch_residual(&c->L, c->L.val, c->r, c->r, nullptr, nullptr, nullptr,
                               c->partials, c->nred, c->red, s));
      GABP_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
      GABP_HIP(hipStreamSynchronize(s));
      return GABP_OK;
    };
    if ((st = time_it(s, 10, one_check, &t_check)) != GABP_OK) return st;
    int ce = 8;
    while (ce < 256 && t_check > 0.02 * ce * t_sweep) ce *= 2;
    t.hints = 0;
    t.block = kBlock;
    t.check_every = ce;
    cache_store(key, t);
    c->fresh64 = true;   // the timing sweeps leave the messages in use: logically zero again
    c->fresh32 = true;
  }
  c->opt.check_every = t.check_every;
  c->graphs->clear();
  if (check_every_out) *check_every_out = t.check_every;
  if (hints_out) *hints_out = 0;
  return GABP_OK;
}

}  // namespace

extern "C" {

int gabp_autotune(gabp_ctx* c, int32_t* check_every_out, int32_t* hints_out,
                  int32_t* block_out, hipStream_t s) {
  if (!c) return fail(GABP_EINVAL, "NULL context");
  if (block_out) *block_out = c->batch || c->lines ? kBlock : c->L.block;
  if (c->lines) return autotune_lines(c, check_every_out, hints_out, s);
  const std::string key = key_of(c);
  Tuned t{};
  const bool f32 = c->opt.precision == GABP_F32_IR;
  bool& hints = f32 ? c->L.stream_hints32 : c->L.stream_hints;
  bool& store_only = f32 ? c->L.store_hints32 : c->L.store_hints;
  if (!cache_lookup(key, &t)) {
    int st;
    const bool seq = c->opt.mode == GABP_MODE_PRECOMP_SEQ;
    // a tiled layout is timed with its two-sweep kernels, the ones its solves launch
    const bool pairs = !c->batch && c->L.ntiles > 0;
    if (seq) {
      if ((st = ensure_seq(c, pairs ? 2 : 1, s)) != GABP_OK) return st;
    } else if (f32 || c->opt.mode == GABP_MODE_PRECOMP) {
      if ((st = precompute(c, 0, s)) != GABP_OK) return st;
    }
    // the mean-only sweeps are timed with the converged Lt, or with the first sweep's Lt
    const double* lam64 = seq ? c->seq.lamout[0] : c->pre[0].lamout;
    const double* S64 = seq ? c->seq.S[0] : c->pre[0].S;
    const float* lam32 = seq ? c->seq.lamout32[0] : c->pre[0].lamout32;
    const float* invS32 = seq ? c->seq.invS32[0] : c->pre[0].invS32;
    const int64_t n = c->L.n;
    const int64_t R = c->batch ? c->batch->R : 1;
    // zero right-hand side and messages: timing only (nothing denormal, nothing non-finite)
    double* zero64 = c->batch ? c->batch->b : c->r;
    GABP_HIP(launch_fill64(zero64, n * R, 0.0, s));
    if (c->batch) {
      GABP_HIP(launch_fill_i32(c->batch->sys_on, c->batch->nsys, 1, s));
      GABP_HIP(launch_fill_i32(c->batch->sys_live, c->batch->nsys, 1, s));
      GABP_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(c->batch->flags),
                               static_cast<int64_t>(c->batch->nsys) * R, 0, s));
      GABP_HIP(launch_fill64(c->batch->x, n * R, 0.0, s));
    }
    float* zero32 = c->batch ? c->batch->r32 : c->r32;
    if (f32) {
      if (!c->msg32[0]) {
        for (int q = 0; q < 2; ++q) {
          GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->msg32[q]), (c->L.epad + 1) * sizeof(float)));
          GABP_HIP(launch_fill32(c->msg32[q], c->L.epad + 1, 0.0f, s));
        }
        GABP_HIP(hipMalloc(reinterpret_cast<void**>(&c->dbest32), c->L.n * sizeof(float)));
      }
      GABP_HIP(launch_fill32(zero32, n * R, 0.0f, s));
    }
    int par = 0;
    auto one_sweep = [&]() -> int {
      Batch* B = c->batch;
      if (pairs) {
        if (f32) {
          MeanPairArgs<float> a{&c->L, lam32, seq ? c->seq.lamout32[1] : lam32,
                                seq ? c->seq.invS32[1] : invS32, zero32, c->msg32[par],
                                c->msg32[par ^ 1], nullptr};
          GABP_HIP(launch_mean_pair32(a, s));
        } else if (c->opt.mode == GABP_MODE_JOINT) {
          SweepArgs a{&c->L, c->L.aT, zero64, c->lam[par], c->msg[par], c->lam[par ^ 1],
                      c->msg[par ^ 1], nullptr, -1};
          GABP_HIP(launch_joint_pair(a, s));
        } else {
          MeanPairArgs<double> a{&c->L, lam64, seq ? c->seq.lamout[1] : lam64,
                                 seq ? c->seq.S[1] : S64, zero64, c->msg[par],
                                 c->msg[par ^ 1], nullptr};
          GABP_HIP(launch_mean_pair64(a, s));
        }
      } else if (B) {
        if (f32) GABP_HIP(batch_mean32(c, B, B->msg32[par], B->msg32[par ^ 1], nullptr, s));
        else if (c->opt.mode == GABP_MODE_JOINT)
          GABP_HIP(batch_joint64(c, B, c->lam[par], B->msg64[par], c->lam[par ^ 1], B->msg64[par ^ 1], nullptr, s));
        else GABP_HIP(batch_mean64(c, B, B->msg64[par], B->msg64[par ^ 1], nullptr, s));
      } else if (f32) {
        MeanArgs32 a{&c->L, lam32, invS32, zero32, c->msg32[par], c->msg32[par ^ 1], nullptr,
                     -1};
        GABP_HIP(launch_mean_sweep32(a, s));
      } else if (c->opt.mode == GABP_MODE_JOINT) {
        SweepArgs a{&c->L, c->L.aT, zero64, c->lam[par], c->msg[par], c->lam[par ^ 1],
                    c->msg[par ^ 1], nullptr, -1};
        GABP_HIP(launch_joint_sweep(a, s));
      } else {
        MeanArgs64 a{&c->L, lam64, S64, zero64, c->msg[par], c->msg[par ^ 1], nullptr, -1};
        GABP_HIP(launch_mean_sweep64(a, s));
      }
      par ^= 1;
      return GABP_OK;
    };
    const int reps = 20;
    double t_sweep = 0.0;
    t.block = kBlock;
    if (c->batch) {   // batched sweeps stream without hints
      if ((st = time_it(s, reps, one_sweep, &t_sweep)) != GABP_OK) return st;
      t.hints = 0;
    } else {
      // every (hints, workgroup size) pair; the fastest is kept (the two-sweep kernels have
      // one workgroup per tile: hints only, per sweep, with the third setting of
      // non-temporal stores and plain loads)
      static const int kBlocks[3] = {64, 128, 256};
      t_sweep = 0.0;
      for (int h = 0; h < (pairs ? 3 : 2); ++h)
        for (int bi = pairs ? 2 : 0; bi < 3; ++bi) {
          hints = h == 1;
          store_only = h == 2;
          c->L.block = kBlocks[bi];
          double tt = 0.0;
          if ((st = time_it(s, reps, one_sweep, &tt)) != GABP_OK) return st;
          if (pairs) tt *= 0.5;
          if (t_sweep == 0.0 || tt < t_sweep) {
            t_sweep = tt;
            t.hints = h;
            t.block = kBlocks[bi];
          }
        }
      hints = t.hints == 1;
      store_only = t.hints == 2;
      c->L.block = t.block;
    }
    // one residual check: residual kernel, reduction, readback and host wait
    double t_check = 0.0;
    auto one_check = [&]() -> int {
      if (c->batch) {
        GABP_HIP(batch_residual(c, c->batch, c->batch->sys_on, c->batch->x, nullptr, nullptr, s));
        GABP_HIP(hipMemcpyAsync(c->batch->host_count, c->batch->count, sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
      } else {
        GABP_HIP(launch_residual(&c->L, c->L.val, zero64, zero64, nullptr, nullptr, nullptr,
                                 c->partials, c->nred, c->red, s));
        GABP_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
      }
      GABP_HIP(hipStreamSynchronize(s));
      return GABP_OK;
    };
    if ((st = time_it(s, 10, one_check, &t_check)) != GABP_OK) return st;
    // smallest power of two that keeps the checks within 2% of the sweep time
    int ce = 8;
    while (ce < 256 && t_check > 0.02 * ce * t_sweep) ce *= 2;
    t.check_every = ce;
    cache_store(key, t);
    c->parity = 0;   // the timing runs leave the buffers in use: logically zero again
    c->parity32 = 0;
    c->fresh64 = true;
    c->fresh32 = true;
  }
  hints = t.hints == 1;
  store_only = t.hints == 2 && c->L.ntiles > 0;
  if (!c->batch) c->L.block = t.block;
  c->opt.check_every = t.check_every;
  c->graphs->clear();
  if (check_every_out) *check_every_out = t.check_every;
  if (hints_out) *hints_out = t.hints;
  if (block_out) *block_out = c->batch ? kBlock : c->L.block;
  return GABP_OK;
}

}  // extern "C"
