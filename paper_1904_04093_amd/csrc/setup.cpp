// Host side of the context: CSR validation, the symmetrised slice layout with its
// reverse-slot index, device allocation and value updates.
//
// Graph construction follows Sec. 2.3: edge j -> i iff A_ij != 0. The layout stores, for
// every row j and every neighbour i of the symmetrised pattern, the message i -> j that j
// receives together with A_ji and A_ij; where only one of the two entries is stored the
// other coefficient is zero, so the message through it is identically zero (Sec. 2.3,
// remark after Algorithm 1), which is how structurally nonsymmetric A is handled.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "gabp_batch.h"
#include "gabp_line.h"
#include "graph.h"

namespace gabp {

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? GABP_ENOMEM : GABP_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

template <typename T>
int upload(T** dst, const std::vector<T>& src, hipStream_t s) {
  const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
  GABP_HIP(hipMalloc(reinterpret_cast<void**>(dst), bytes));
  if (!src.empty())
    GABP_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return GABP_OK;
}

template <typename T>
int alloc(T** dst, int64_t count) {
  const size_t bytes = static_cast<size_t>(std::max<int64_t>(count, 1)) * sizeof(T);
  GABP_HIP(hipMalloc(reinterpret_cast<void**>(dst), bytes));
  return GABP_OK;
}

}  // namespace
}  // namespace gabp

using namespace gabp;

extern "C" {

void gabp_default_options(gabp_options* o) {
  if (!o) return;
  o->mode = GABP_MODE_JOINT;
  o->precision = GABP_F64;
  o->check_every = 16;
  o->tol_lambda = 1e-14;
  o->max_lambda_sweeps = 100000;
  o->ir_inner_tol = 1e-4;
  o->ir_max_inner = 1000000;
  o->schedule = GABP_SCHED_FLOOD;
  o->use_graphs = 1;
  o->grid_nx = 0;
  o->grid_ny = 0;
  o->block = kBlock;
  o->tiles = 0;
  o->progress_s = 0.0;
  o->stream_hints = -1;
}


int gabp_setup(gabp_ctx** out, int32_t n, int64_t nnz, const int32_t* rowptr,
               const int32_t* col, const double* val, const int32_t* rev,
               const uint8_t* colour, const gabp_options* opt, hipStream_t stream) {
  if (!out) return fail(GABP_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate(n, nnz, rowptr, col, val, rev);
  if (st != GABP_OK) return st;
  gabp_options o;
  gabp_default_options(&o);
  if (opt) o = *opt;
  if (o.check_every < 1 || o.max_lambda_sweeps < 0 || o.tol_lambda < 0 ||
      (o.mode < GABP_MODE_JOINT || o.mode > GABP_MODE_PRECOMP_SEQ) ||
      (o.precision != GABP_F64 && o.precision != GABP_F32_IR) ||
      (o.schedule < GABP_SCHED_FLOOD || o.schedule > GABP_SCHED_LINES_ALT) ||
      o.ir_max_inner < 1 || !(o.progress_s >= 0.0) ||
      (o.block != 64 && o.block != 128 && o.block != 256) || (o.tiles != 0 && o.tiles != 1) ||
      !(o.ir_inner_tol > 0.0) || o.stream_hints < -1 || o.stream_hints > 2)
    return fail(GABP_EINVAL, "invalid options");
  if (o.stream_hints == 2 && !o.tiles)
    return fail(GABP_EINVAL, "stream_hints 2 (non-temporal stores only) needs a tiled layout");
  if (o.schedule == GABP_SCHED_REDBLACK && !colour)
    return fail(GABP_EINVAL, "red-black schedule needs node colours");
  if (o.mode == GABP_MODE_PRECOMP_SEQ &&
      (o.schedule == GABP_SCHED_LINES || o.schedule == GABP_SCHED_LINES_ALT))
    return fail(GABP_ENOTSUPP, "per-sweep precision messages are built for point schedules");
  int32_t inject_at = -1;
  bool poison = false;
  if (const char* fi = std::getenv("GABP_FAULT_INJECT")) {
    int k = -1;
    char tail = 0;
    if (std::strcmp(fi, "poison-outputs") == 0)
      poison = true;
    else if (std::sscanf(fi, "nan@sweep:%d%c", &k, &tail) == 1 && k >= 0)
      inject_at = k;
    else
      return fail(GABP_EINVAL, "GABP_FAULT_INJECT must read nan@sweep:<k> (k >= 0) or "
                               "poison-outputs");
  }

  // --- transposed pattern (counting sort): tptr/trow/tidx list entries (i, j) by column j
  std::vector<int64_t> tptr(n + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) tptr[col[e] + 1]++;
  for (int32_t j = 0; j < n; ++j) tptr[j + 1] += tptr[j];
  std::vector<int32_t> trow(nnz), tidx(nnz);
  {
    std::vector<int64_t> cur(tptr.begin(), tptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int64_t q = cur[col[e]]++;
        trow[q] = i;
        tidx[q] = static_cast<int32_t>(e);
      }
  }
  // --- symmetrised off-diagonal pattern of every row (merge of row j and column j)
  std::vector<int64_t> uptr(n + 1, 0);
  std::vector<int32_t> unbr, uval, uaT;   // neighbour, CSR index of A_ji, CSR index of A_ij
  unbr.reserve(static_cast<size_t>(nnz) * 2);
  uval.reserve(static_cast<size_t>(nnz) * 2);
  uaT.reserve(static_cast<size_t>(nnz) * 2);
  std::vector<int32_t> diag_src(n, -1);
  int32_t max_w = 0;
  for (int32_t j = 0; j < n; ++j) {
    int64_t a = rowptr[j], ae = rowptr[j + 1];
    int64_t t = tptr[j], te = tptr[j + 1];
    int32_t w = 0;
    while (a < ae || t < te) {
      const int32_t ca = a < ae ? col[a] : std::numeric_limits<int32_t>::max();
      const int32_t ct = t < te ? trow[t] : std::numeric_limits<int32_t>::max();
      const int32_t c = std::min(ca, ct);
      int32_t iv = -1, ia = -1;
      if (ca == c) iv = static_cast<int32_t>(a++);
      if (ct == c) ia = tidx[t++];
      if (c == j) {
        diag_src[j] = iv;
        continue;
      }
      unbr.push_back(c);
      uval.push_back(iv);
      uaT.push_back(ia);
      ++w;
    }
    uptr[j + 1] = uptr[j] + w;
    max_w = std::max(max_w, w);
  }
  const int64_t slots = uptr[n];
  // --- lanes: row j at lane j, or (with colours) colour-major: the rows of each colour in
  // ascending order, each colour padded to whole slices; lanes without a row hold -1
  std::vector<int32_t> lane_of_row, row_of_lane, cstart;
  int ncolours = 0;
  int64_t nlanes = n;
  if (colour) {
    for (int32_t j = 0; j < n; ++j) {
      if (colour[j] >= kMaxColours)
        return fail(GABP_EINVAL, "colour must be below " + std::to_string(kMaxColours));
      ncolours = std::max(ncolours, colour[j] + 1);
    }
    std::vector<int64_t> cnt(ncolours, 0), next(ncolours);
    for (int32_t j = 0; j < n; ++j) ++cnt[colour[j]];
    // every class starts on a slice boundary: a class launch's wavefronts then each lie in
    // one slice, which the sweep kernels rely on (they read a wavefront's slot range once)
    int64_t acc = 0;
    for (int c = 0; c < ncolours; ++c) {
      next[c] = acc;
      acc += (cnt[c] + kSlice - 1) / kSlice * kSlice;
    }
    if (acc >= std::numeric_limits<int32_t>::max() - kBlock)
      return fail(GABP_ENOTSUPP, "too many rows for a coloured layout");
    cstart.assign(ncolours + 1, static_cast<int32_t>(acc));
    for (int c = 0; c < ncolours; ++c) cstart[c] = static_cast<int32_t>(next[c]);
    nlanes = acc;
    lane_of_row.resize(n);
    row_of_lane.assign(static_cast<size_t>(nlanes), -1);
    for (int32_t j = 0; j < n; ++j) {
      const int64_t t = next[colour[j]]++;
      lane_of_row[j] = static_cast<int32_t>(t);
      row_of_lane[t] = j;
    }
  }
  // --- tiles (temporal blocking, flood schedule on a grid): lanes tile-major, each tile
  // tsl slices of 64 x-consecutive nodes of tsl consecutive grid rows,
  // padded with empty lanes past the grid's right and top edges
  const bool tiled = o.tiles != 0;
  // FP64 sweeps: one lane per thread (more registers per lane would halve the workgroups
  // per CU); FP32 mean-only sweeps: two lanes per thread, twice the tile and half the
  // halo per row
  const int32_t tsl = o.precision == GABP_F32_IR ? 2 * kTileUnit : kTileUnit;
  int32_t tiles_x = 0, tiles_y = 0;
  if (tiled) {
    if (colour || o.schedule != GABP_SCHED_FLOOD)
      return fail(GABP_EINVAL, "tiles need the flood schedule (no colouring)");
    if (o.grid_nx < 1 || o.grid_ny < 1 || static_cast<int64_t>(o.grid_nx) * o.grid_ny != n)
      return fail(GABP_EINVAL, "tiles need grid_nx * grid_ny == n");
    if (max_w > kTileMaxWidth)
      return fail(GABP_ENOTSUPP, "tiles need rows of at most " + std::to_string(kTileMaxWidth) +
                                     " off-diagonal neighbours (5-point grids)");
    tiles_x = (o.grid_nx + kSlice - 1) / kSlice;
    tiles_y = (o.grid_ny + tsl - 1) / tsl;
    nlanes = static_cast<int64_t>(tiles_x) * tiles_y * tsl * kSlice;
    if (nlanes >= std::numeric_limits<int32_t>::max() - kBlock)
      return fail(GABP_ENOTSUPP, "too many rows for a tiled layout");
    lane_of_row.assign(n, -1);
    row_of_lane.assign(static_cast<size_t>(nlanes), -1);
    for (int32_t ty = 0; ty < tiles_y; ++ty)
      for (int32_t tx = 0; tx < tiles_x; ++tx)
        for (int32_t r = 0; r < tsl; ++r)
          for (int32_t cx = 0; cx < kSlice; ++cx) {
            const int64_t x = static_cast<int64_t>(tx) * kSlice + cx;
            const int64_t y = static_cast<int64_t>(ty) * tsl + r;
            if (x >= o.grid_nx || y >= o.grid_ny) continue;
            const int64_t t = ((static_cast<int64_t>(ty) * tiles_x + tx) * tsl + r) * kSlice + cx;
            const int32_t j = static_cast<int32_t>(y * o.grid_nx + x);
            lane_of_row[j] = static_cast<int32_t>(t);
            row_of_lane[t] = j;
          }
  }
  auto row_at = [&](int64_t t) -> int32_t {
    return !row_of_lane.empty() ? row_of_lane[t] : (t < n ? static_cast<int32_t>(t) : -1);
  };
  // --- slices of 64 lanes, column-major inside a slice
  const int32_t nslices = static_cast<int32_t>((nlanes + kSlice - 1) / kSlice);
  std::vector<int64_t> sptr64(nslices + 1, 0);
  for (int32_t s = 0; s < nslices; ++s) {
    int64_t w = 0;
    for (int64_t t = static_cast<int64_t>(s) * kSlice; t < std::min<int64_t>(nlanes, (s + 1) * int64_t(kSlice)); ++t) {
      const int32_t j = row_at(t);
      if (j >= 0) w = std::max<int64_t>(w, uptr[j + 1] - uptr[j]);
    }
    sptr64[s + 1] = sptr64[s] + w * kSlice;
  }
  const int64_t epad = sptr64[nslices];
  if (epad + 1 >= std::numeric_limits<int32_t>::max())
    return fail(GABP_ENOTSUPP, "more than 2^31-1 padded message slots");
  auto pos = [&](int32_t j, int64_t k) -> int64_t {   // slot k of row j
    const int64_t t = lane_of_row.empty() ? j : lane_of_row[j];
    return sptr64[t / kSlice] + k * kSlice + t % kSlice;
  };
  // padding slots are their own reverse: every sweep writes a zero message there, so each
  // slot a sweep reads was written by the sweep before (or the reset)
  std::vector<int32_t> h_rev(epad), h_col(epad, 0);
  for (int64_t p = 0; p < epad; ++p) h_rev[p] = static_cast<int32_t>(p);
  std::vector<int32_t> h_vsrc(epad, -1), h_asrc(epad, -1);
  std::vector<double> h_val(epad, 0.0), h_aT(epad, 0.0), h_diag(n);
  for (int32_t s = 0; s < nslices; ++s) {   // padding slots: own row as column (coef 0)
    const int64_t w = (sptr64[s + 1] - sptr64[s]) / kSlice;
    for (int32_t lane = 0; lane < kSlice; ++lane)
      for (int64_t k = 0; k < w; ++k)
        h_col[sptr64[s] + k * kSlice + lane] = std::min(n - 1, s * kSlice + lane);
  }
  std::vector<int64_t> cursor(uptr.begin(), uptr.end() - 1);
  for (int32_t j = 0; j < n; ++j) {
    h_diag[j] = val[diag_src[j]];
    for (int64_t k = 0; k < uptr[j + 1] - uptr[j]; ++k) {
      const int64_t u = uptr[j] + k;
      const int32_t i = unbr[u];
      const int64_t p = pos(j, k);
      // rows are visited in ascending j and every row lists its neighbours ascending, so
      // the next unvisited slot of row i is (i, j)
      const int64_t ui = cursor[i]++;
      if (unbr[ui] != j) return fail(GABP_EINVAL, "internal: asymmetric union pattern");
      h_rev[p] = static_cast<int32_t>(pos(i, ui - uptr[i]));
      h_col[p] = i;
      h_vsrc[p] = uval[u];
      h_asrc[p] = uaT[u];
      h_val[p] = uval[u] >= 0 ? val[uval[u]] : 0.0;
      h_aT[p] = uaT[u] >= 0 ? val[uaT[u]] : 0.0;
    }
  }
  if (colour) {
    for (int32_t j = 0; j < n; ++j) {
      for (int64_t u = uptr[j]; u < uptr[j + 1]; ++u)
        if (colour[unbr[u]] == colour[j])
          return fail(GABP_EINVAL, "colouring is not proper: edge inside one colour at row " +
                                       std::to_string(j));
    }
  }
  // int16 reverse deltas when every real slot's reverse is within +-32767 positions
  std::vector<int16_t> h_rev16;
  bool rev16_classed = false;
  {
    bool fits = true;
    for (int64_t p = 0; p < epad && fits; ++p) {
      const int64_t d = static_cast<int64_t>(h_rev[p]) - p;
      fits = d >= -32767 && d <= 32767;
    }
    if (fits) {
      h_rev16.resize(epad);
      for (int64_t p = 0; p < epad; ++p) h_rev16[p] = static_cast<int16_t>(h_rev[p] - p);
    } else if (colour && ncolours == 2) {
      // two colour classes: a real slot's reverse lies in the other class at about the same
      // relative position, so the delta is taken from the other class's first slot
      const int64_t cs1 = sptr64[cstart[1] / kSlice];
      bool ok = true;
      std::vector<int16_t> d16(epad);
      for (int64_t p = 0; p < epad && ok; ++p) {
        if (h_rev[p] == p) {
          d16[p] = static_cast<int16_t>(kRevSelf16);
          continue;
        }
        const int64_t shift = p < cs1 ? cs1 : -cs1;
        const int64_t d = static_cast<int64_t>(h_rev[p]) - p - shift;
        ok = d >= -32767 && d <= 32767;
        d16[p] = static_cast<int16_t>(d);
      }
      if (ok) {
        h_rev16.swap(d16);
        rev16_classed = true;
      }
    }
  }
  std::vector<int32_t> h_sptr(nslices + 1);
  for (int32_t s = 0; s <= nslices; ++s) h_sptr[s] = static_cast<int32_t>(sptr64[s]);
  std::vector<int32_t> h_row(nnz), h_ccol(col, col + nnz);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) h_row[e] = i;

  gabp_ctx* c = new gabp_ctx();
  c->opt = o;
  c->inject_nan_at = inject_at;
  c->poison_outputs = poison;
  c->graphs = new GraphCache();
  GABP_HIP(hipGetDevice(&c->device));
  Layout& L = c->L;
  L.n = n;
  L.nnz = nnz;
  L.slots = slots;
  L.epad = epad;
  L.nslices = nslices;
  L.nlanes = static_cast<int32_t>(nlanes);
  L.max_width = max_w;
  L.block = o.block;
  // footprint of one FP64 joint sweep (44 B per slot, 16 B per row) and one FP32 mean
  // sweep (16 B per slot, 4 B per row) against the 256 MiB last-level cache
  constexpr double kLLC = 256.0 * 1024 * 1024;
  L.stream_hints = 44.0 * epad + 16.0 * n > kLLC;
  L.stream_hints32 = 16.0 * epad + 4.0 * n > 2.0 * kLLC;
  // residual: 12 B per slot (column, coefficient) + 32 B per row (row slot, b, diag, x, r)
  L.res_hints = 12.0 * epad + 32.0 * n > kLLC;
  if (o.stream_hints >= 0) {
    L.stream_hints = L.stream_hints32 = o.stream_hints == 1;
    L.store_hints = L.store_hints32 = o.stream_hints == 2;
  }
  auto cleanup_fail = [&](int code) {
    gabp_destroy(c);
    return code;
  };
#define UP(dst, src) \
  if ((st = upload(&(dst), src, stream)) != GABP_OK) return cleanup_fail(st)
#define AL(dst, cnt) \
  if ((st = alloc(&(dst), cnt)) != GABP_OK) return cleanup_fail(st)
  if ((st = scratch_on(c->device, nullptr)) != GABP_OK) return cleanup_fail(st);
  UP(L.sptr, h_sptr);
  UP(L.rev, h_rev);
  if (!h_rev16.empty()) UP(L.rev16, h_rev16);
  L.rev16_classed = rev16_classed;
  UP(L.col, h_col);
  UP(L.val, h_val);
  UP(L.aT, h_aT);
  UP(L.diag, h_diag);
  UP(L.val_src, h_vsrc);
  UP(L.aT_src, h_asrc);
  UP(L.diag_src, diag_src);
  UP(L.csr_row, h_row);
  UP(L.csr_col, h_ccol);
  std::vector<int32_t> row_slot;
  if (epad < (int64_t(1) << kRowSlotShift) && max_w < (1 << (32 - kRowSlotShift))) {
    row_slot.resize(n);
    for (int32_t j = 0; j < n; ++j) {
      const int64_t t = lane_of_row.empty() ? j : lane_of_row[j];
      const int64_t sl = t / kSlice;
      const int64_t w = (sptr64[sl + 1] - sptr64[sl]) / kSlice;
      row_slot[j] = static_cast<int32_t>((sptr64[sl] + t % kSlice) | (w << kRowSlotShift));
    }
    UP(L.row_slot, row_slot);
  }
  if (!row_of_lane.empty()) {
    UP(L.perm, row_of_lane);
    UP(L.lane_of_row_d, lane_of_row);
    L.lane_of_row = lane_of_row;
  }
  // (kept until the end of set-up: the uploads below are asynchronous)
  std::vector<int32_t> hptr, hlane;
  std::vector<int4> halo;
  if (tiled) {
    // halo of each tile: the rows outside it that send into it (neighbours of its rows in
    // the symmetrised pattern), in ascending lane order, each as {first slot, slots, row}
    const int32_t ntiles = tiles_x * tiles_y;
    hptr.assign(ntiles + 1, 0);
    std::vector<int32_t> mark(static_cast<size_t>(nlanes), -1);
    int32_t slots_max = 0;
    for (int32_t t = 0; t < ntiles; ++t) {
      const int64_t l0 = static_cast<int64_t>(t) * tsl * kSlice;
      const int64_t l1 = l0 + tsl * kSlice;
      std::vector<int32_t> h;
      for (int64_t ln = l0; ln < l1; ++ln) {
        const int32_t j = row_of_lane[ln];
        if (j < 0) continue;
        for (int64_t u = uptr[j]; u < uptr[j + 1]; ++u) {
          const int32_t li = lane_of_row[unbr[u]];
          if ((li < l0 || li >= l1) && mark[li] != t) {
            mark[li] = t;
            h.push_back(li);
          }
        }
      }
      std::sort(h.begin(), h.end());
      hlane.insert(hlane.end(), h.begin(), h.end());
      hptr[t + 1] = static_cast<int32_t>(hlane.size());
      slots_max = std::max<int32_t>(
          slots_max, static_cast<int32_t>(sptr64[(t + 1) * tsl] - sptr64[t * tsl]));
    }
    // one entry per halo thread of each tile's workgroup, {first slot, slots, row, 0}
    halo.assign(static_cast<size_t>(ntiles) * kHaloThreads, int4{0, 0, 0, 0});
    for (int32_t t = 0; t < ntiles; ++t) {
      if (hptr[t + 1] - hptr[t] > kHaloThreads)
        return cleanup_fail(fail(GABP_ENOTSUPP, "a tile's halo exceeds " +
                                                    std::to_string(kHaloThreads) + " rows"));
      for (int32_t q = hptr[t]; q < hptr[t + 1]; ++q) {
        const int64_t ln = hlane[q];
        const int64_t sl = ln / kSlice;
        halo[static_cast<size_t>(t) * kHaloThreads + (q - hptr[t])] =
            int4{static_cast<int32_t>(sptr64[sl] + ln % kSlice),
                 static_cast<int32_t>((sptr64[sl + 1] - sptr64[sl]) / kSlice), row_of_lane[ln], 0};
      }
    }
    UP(L.tile_halo, halo);
    L.ntiles = ntiles;
    L.tiles_x = tiles_x;
    L.grid_nx = o.grid_nx;
    L.grid_ny = o.grid_ny;
    // XCD-aware tile order: one strip of tile columns per XCD where the width allows
    L.tile_strip = std::max<int32_t>(1, (tiles_x + kXcds - 1) / kXcds);
    L.tile_slices = tsl;
    L.tile_slots_max = slots_max;
  }
  if (colour) {
    L.ncolours = ncolours;
    L.cstart = cstart;
    L.cslot.resize(cstart.size());
    for (size_t q = 0; q < cstart.size(); ++q)
      L.cslot[q] = static_cast<int32_t>(sptr64[cstart[q] / kSlice]);
  }
  {   // FNV-1a over the slot and lane layout: two contexts share message positions iff equal
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](int64_t v) {
      for (int q = 0; q < 8; ++q) {
        h ^= static_cast<uint64_t>(v >> (8 * q)) & 0xffu;
        h *= 1099511628211ull;
      }
    };
    mix(n); mix(epad); mix(nlanes); mix(ncolours); mix(tiled ? 1 : 0);
    for (int32_t q = 0; q <= nslices; ++q) mix(sptr64[q]);
    for (int32_t t : lane_of_row) mix(t);
    L.hash = h;
  }
  for (int q = 0; q < 2; ++q) {
    AL(c->lam[q], epad + 1);
    AL(c->msg[q], epad + 1);
  }
  AL(c->r, n);
  AL(c->r2, n);
  AL(c->e, n);
  AL(c->r32, n);
  AL(c->d32, n);
  c->nred = static_cast<int32_t>((nlanes + kRedBlock - 1) / kRedBlock);
  c->npartials = std::max<int64_t>(3 * static_cast<int64_t>(c->nred),
                                   2 * ((nlanes + kBlock - 1) / kBlock));
  AL(c->partials, c->npartials);
  AL(c->red, 8);
  AL(c->lmax, 2);
#undef UP
#undef AL
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_red), 8 * sizeof(double),
                    hipHostMallocDefault) != hipSuccess)
    return cleanup_fail(fail(GABP_ENOMEM, "pinned host buffer"));
  for (int q = 0; q < 2; ++q) {
    hipError_t e1 = launch_fill64(c->lam[q], epad + 1, 0.0, stream);
    hipError_t e2 = launch_fill64(c->msg[q], epad + 1, 0.0, stream);
    if (e1 != hipSuccess || e2 != hipSuccess) return cleanup_fail(hip_fail(e1 != hipSuccess ? e1 : e2, "fill"));
  }
  if (o.schedule == GABP_SCHED_LINES || o.schedule == GABP_SCHED_LINES_ALT) {
    const int lst = line_setup(c, o.grid_nx, o.grid_ny, rowptr, col, val);
    if (lst != GABP_OK) return cleanup_fail(lst);
  }
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return cleanup_fail(hip_fail(e, "hipStreamSynchronize(setup)"));
  *out = c;
  return GABP_OK;
}

int gabp_update_values(gabp_ctx* c, const double* val, hipStream_t stream) {
  if (!c || !val) return fail(GABP_EINVAL, "NULL argument");
  int* bad = reinterpret_cast<int*>(c->lmax);   // reuse 16 bytes of scratch as a flag
  GABP_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
  GABP_HIP(launch_update_values(&c->L, val, bad, stream));
  if (c->lines) {
    const int lst = line_update_values(c, val, stream);
    if (lst != GABP_OK) return lst;
  }
  int hbad = 0;
  GABP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  GABP_HIP(hipStreamSynchronize(stream));
  // recorded blocks read the coefficient and precomputed-Lt buffers in place, so they stay
  // valid; only the precomputed Lt must be recomputed for the new values
  c->pre[0].valid = c->pre[1].valid = false;
  c->seq.valid = false;
  if (hbad) return fail(GABP_EZERODIAG, "zero or non-finite diagonal in updated values");
  return GABP_OK;
}

void gabp_destroy(gabp_ctx* c) {
  if (!c) return;
  auto F = [](void* p) {
    if (p) (void)hipFree(p);
  };
  Layout& L = c->L;
  F(L.sptr); F(L.rev); F(L.rev16); F(L.col); F(L.val); F(L.aT); F(L.diag); F(L.val_src); F(L.aT_src);
  F(L.diag_src); F(L.csr_row); F(L.csr_col); F(L.perm); F(L.lane_of_row_d);
  F(L.tile_halo); F(L.row_slot);
  for (int q = 0; q < 2; ++q) {
    F(c->lam[q]); F(c->msg[q]); F(c->msg32[q]);
    F(c->pre[q].lamout); F(c->pre[q].S); F(c->pre[q].lamout32); F(c->pre[q].invS32);
  }
  free_seq(c);
  F(c->r); F(c->r2); F(c->e); F(c->bsol); F(c->xsol); F(c->r32); F(c->d32); F(c->dbest32); F(c->partials); F(c->red); F(c->lmax);
  if (c->host_red) (void)hipHostFree(c->host_red);
  if (c->batch) {
    batch_free(c->batch);
    delete c->batch;
  }
  line_destroy(c->lines);
  delete c->graphs;
  delete c;
}

int gabp_layout_info(const gabp_ctx* c, int32_t* n, int64_t* nnz, int64_t* slots,
                     int64_t* padded, int32_t* rev_bytes) {
  if (!c) return fail(GABP_EINVAL, "NULL context");
  if (n) *n = c->L.n;
  if (nnz) *nnz = c->L.nnz;
  if (slots) *slots = c->L.slots;
  if (padded) *padded = c->L.epad;
  if (rev_bytes) *rev_bytes = c->L.rev16 ? 2 : 4;
  return GABP_OK;
}

}  // extern "C"
