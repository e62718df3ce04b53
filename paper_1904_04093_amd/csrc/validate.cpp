// Host-only part of the library: status texts, the last-error message and the CSR check
// behind gabp_validate_csr / gabp_setup. No device code and no HIP runtime call, so it
// also builds with a plain host compiler (the address-sanitizer test does that).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/gabp.h"

namespace gabp {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// The matrix of Sec. 2.3: every row stores its diagonal (finite, nonzero) and its other
// entries with strictly increasing columns; rev (optional) pairs entry (i, j) with (j, i).
// rowptr is checked whole before any column is read, so a malformed rowptr cannot make the
// check read past col / val.
int validate(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
             const double* val, const int32_t* rev) {
  if (n <= 0) return fail(GABP_EINVAL, "n must be positive");
  if (!rowptr || !col || !val) return fail(GABP_EINVAL, "NULL CSR array");
  if (nnz < n) return fail(GABP_EINVAL, "nnz < n: the diagonal must be stored");
  if (rowptr[0] != 0 || rowptr[n] != nnz) return fail(GABP_EINVAL, "rowptr[0] != 0 or rowptr[n] != nnz");
  for (int32_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i] || rowptr[i + 1] > nnz)
      return fail(GABP_EINVAL, "rowptr not monotone within [0, nnz] at row " + std::to_string(i));
  for (int32_t i = 0; i < n; ++i) {
    bool has_diag = false;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int32_t c = col[e];
      if (c < 0 || c >= n) return fail(GABP_EINVAL, "column out of range in row " + std::to_string(i));
      if (e > rowptr[i] && col[e - 1] >= c)
        return fail(GABP_EINVAL, "columns not strictly increasing in row " + std::to_string(i));
      if (!std::isfinite(val[e])) return fail(GABP_EINVAL, "non-finite value in row " + std::to_string(i));
      if (c == i) {
        has_diag = true;
        if (val[e] == 0.0) return fail(GABP_EZERODIAG, "zero diagonal at row " + std::to_string(i));
      }
    }
    if (!has_diag) return fail(GABP_EZERODIAG, "missing diagonal at row " + std::to_string(i));
  }
  if (rev) {
    std::vector<int32_t> row_of(static_cast<size_t>(nnz));
    for (int32_t i = 0; i < n; ++i)
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) row_of[e] = i;
    for (int32_t i = 0; i < n; ++i) {
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int32_t j = col[e];
        const int64_t r = rev[e];
        // locate (j, i) by binary search
        const int32_t* b = col + rowptr[j];
        const int32_t* en = col + rowptr[j + 1];
        const int32_t* f = std::lower_bound(b, en, i);
        const int64_t expect = (f != en && *f == i) ? (f - col) : -1;
        if (j == i) {
          if (r != e && r != -1) return fail(GABP_EINVAL, "rev of a diagonal entry must be itself or -1");
          continue;
        }
        if (r != expect) return fail(GABP_EINVAL, "rev inconsistent at entry " + std::to_string(e));
        if (r >= 0 && (row_of[r] != j || col[r] != i))
          return fail(GABP_EINVAL, "rev does not point at the transposed entry");
      }
    }
  }
  return GABP_OK;
}

}  // namespace gabp

extern "C" {

const char* gabp_strerror(int s) {
  switch (s) {
    case GABP_OK: return "ok";
    case GABP_MAXSWEEPS: return "tolerance not reached within max_sweeps";
    case GABP_EINVAL: return "invalid argument";
    case GABP_ENOMEM: return "out of memory";
    case GABP_EZERODIAG: return "missing or zero diagonal entry";
    case GABP_ENUMERIC: return "non-finite value (zero cavity precision or divergence)";
    case GABP_EDEVICE: return "HIP runtime error";
    case GABP_ENOTSUPP: return "not supported";
    default: return "unknown status";
  }
}

const char* gabp_last_error(void) { return gabp::g_last_error.c_str(); }

int gabp_validate_csr(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                      const double* val, const int32_t* rev) {
  return gabp::validate(n, nnz, rowptr, col, val, rev);
}

}  // extern "C"
