// Status codes, thread-local error messages and host-side CSR validation.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.hpp"

namespace cpra {

static thread_local char g_msg[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
}

void clear_error() { g_msg[0] = '\0'; }

cpra_status check_csr(const cpra_csr* g, const char* who, bool need_inv_deg, bool need_wdeg) {
  if (g == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "%s: graph is NULL", who);
  if (g->n_nodes < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "%s: n_nodes = %d < 0", who, g->n_nodes);
  if (g->nnz < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "%s: nnz < 0", who);
  if (g->nnz >= (int64_t(1) << 31))
    CPRA_FAIL(CPRA_ERR_OVERFLOW, "%s: nnz = %lld does not fit int32 indexing", who,
              (long long)g->nnz);
  if (g->n_graphs < 1) CPRA_FAIL(CPRA_ERR_SHAPE, "%s: n_graphs = %d < 1", who, g->n_graphs);
  if (g->n_graphs > 1 && g->graph_ptr == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "%s: graph_ptr is NULL with n_graphs = %d", who, g->n_graphs);
  if (g->n_graphs == 1 && g->graph_ptr != nullptr)
    CPRA_FAIL(CPRA_ERR_SHAPE, "%s: graph_ptr must be NULL when n_graphs == 1", who);
  if (g->n_nodes > 0 && g->row_ptr == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "%s: row_ptr is NULL", who);
  if (g->nnz > 0 && g->col_idx == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "%s: col_idx is NULL", who);
  if (need_inv_deg && g->n_nodes > 0 && g->inv_deg == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "%s: inv_deg is NULL (run cpra_csr_prepare)", who);
  if (need_wdeg && g->n_nodes > 0 && g->wdeg == nullptr)
    CPRA_FAIL(CPRA_ERR_NULL, "%s: wdeg is NULL (run cpra_csr_prepare)", who);
  return CPRA_OK;
}

}  // namespace cpra

extern "C" {

int32_t cpra_abi_version(void) { return CPRA_ABI_VERSION; }

const char* cpra_status_string(cpra_status s) {
  switch (s) {
    case CPRA_OK: return "CPRA_OK";
    case CPRA_ERR_NULL: return "CPRA_ERR_NULL";
    case CPRA_ERR_SHAPE: return "CPRA_ERR_SHAPE";
    case CPRA_ERR_CSR: return "CPRA_ERR_CSR";
    case CPRA_ERR_PARAM: return "CPRA_ERR_PARAM";
    case CPRA_ERR_OVERFLOW: return "CPRA_ERR_OVERFLOW";
    case CPRA_ERR_WORKSPACE: return "CPRA_ERR_WORKSPACE";
    case CPRA_ERR_HIP: return "CPRA_ERR_HIP";
    case CPRA_ERR_NONFINITE: return "CPRA_ERR_NONFINITE";
  }
  return "CPRA_ERR_UNKNOWN";
}

const char* cpra_last_error_message(void) { return cpra::g_msg; }

cpra_status cpra_csr_validate_host(int32_t n, int64_t nnz, const int32_t* row_ptr,
                                   const int32_t* col_idx, const float* weight) {
  using cpra::set_error;
  if (n < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "validate: n_nodes < 0");
  if (nnz < 0) CPRA_FAIL(CPRA_ERR_SHAPE, "validate: nnz < 0");
  if (nnz >= (int64_t(1) << 31)) CPRA_FAIL(CPRA_ERR_OVERFLOW, "validate: nnz >= 2^31");
  if (row_ptr == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "validate: row_ptr is NULL");
  if (nnz > 0 && col_idx == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "validate: col_idx is NULL");
  if (row_ptr[0] != 0) CPRA_FAIL(CPRA_ERR_CSR, "validate: row_ptr[0] = %d != 0", row_ptr[0]);
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i])
      CPRA_FAIL(CPRA_ERR_CSR, "validate: row_ptr decreases at row %d", i);
  if (row_ptr[n] != nnz)
    CPRA_FAIL(CPRA_ERR_CSR, "validate: row_ptr[N] = %d != nnz = %lld", row_ptr[n], (long long)nnz);
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t j = col_idx[k];
      if (j < 0 || j >= n) CPRA_FAIL(CPRA_ERR_CSR, "validate: row %d has column %d out of range", i, j);
      if (j == i) CPRA_FAIL(CPRA_ERR_CSR, "validate: self loop at node %d", i);
      if (k > row_ptr[i] && col_idx[k - 1] >= j)
        CPRA_FAIL(CPRA_ERR_CSR, "validate: row %d is not strictly increasing", i);
      if (weight && !std::isfinite(weight[k]))
        CPRA_FAIL(CPRA_ERR_NONFINITE, "validate: weight of entry (%d,%d) is not finite", i, j);
    }
  }
  // symmetry: for each (i, j) find i in row j by binary search
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t j = col_idx[k];
      const int32_t* b = col_idx + row_ptr[j];
      const int32_t* e = col_idx + row_ptr[j + 1];
      const int32_t* f = std::lower_bound(b, e, i);
      if (f == e || *f != i)
        CPRA_FAIL(CPRA_ERR_CSR, "validate: entry (%d,%d) has no mirror (%d,%d)", i, j, j, i);
      if (weight && weight[k] != weight[f - col_idx])
        CPRA_FAIL(CPRA_ERR_CSR, "validate: weight of (%d,%d) differs from (%d,%d)", i, j, j, i);
    }
  }
  cpra::clear_error();
  return CPRA_OK;
}

}  // extern "C"
