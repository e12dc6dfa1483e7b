// C ABI of libfinger: argument checking, handle lifetime, workspace layout
// and the order of kernel launches.  Every entry point returns a status and
// records a message for finger_last_error(); no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/finger.h"
#include "internal.h"
#include "abi_util.h"

using finger::Tables;
using finger::rpad_of;

using namespace finger::abi;

extern "C" {

const char* finger_last_error(void) { return g_err.c_str(); }

void finger_build_params_init(finger_build_params* p) {
  if (p == nullptr) return;
  std::memset(p, 0, sizeof(*p));
  p->rank = 0;
  p->code_type = FINGER_CODE_F32;
  p->metric = FINGER_L2;
  p->sigma_mode = FINGER_SIGMA_STD;
  p->n_samples = 0;
  p->seed = 0;
  p->pivots = nullptr;
  p->n_pivots = 0;
  p->dm_override = 0;
}

void finger_search_params_init(finger_search_params* p) {
  if (p == nullptr) return;
  std::memset(p, 0, sizeof(*p));
  p->mode = FINGER_MODE_PLAIN;
  p->k = 10;
  p->ef = 64;
  p->entry = 0;
  p->warmup = 5;
  p->k_max = 0;
  p->ef_max = 0;
  p->persistent = 0;
}

int finger_build_tables(const float* data, int64_t n, int32_t m, const int32_t* graph,
                        int32_t max_degree, const finger_build_params* p, finger_tables** out,
                        void* stream) {
  using namespace finger;
  if (out == nullptr) return fail(FINGER_EINVAL, "out is NULL");
  *out = nullptr;
  if (p == nullptr) return fail(FINGER_EINVAL, "params is NULL");
  if (data == nullptr) return fail(FINGER_EINVAL, "data is NULL");
  if (graph == nullptr) return fail(FINGER_EINVAL, "graph is NULL");
  if (n <= 0 || n >= (int64_t)1 << 31) return fail(FINGER_EINVAL, "n = %lld out of range [1, 2^31)", (long long)n);
  if (m <= 0 || m > kMaxDim || m % 4 != 0)
    return fail(FINGER_EINVAL, "m = %d must be a multiple of 4 in [4, %d]", m, kMaxDim);
  if ((reinterpret_cast<uintptr_t>(data) & 15u) != 0) return fail(FINGER_EINVAL, "data must be 16-byte aligned");
  if (max_degree < 1 || max_degree > kMaxDegree)
    return fail(FINGER_EINVAL, "max_degree = %d out of range [1, %d]", max_degree, kMaxDegree);
  if (p->rank < 0 || p->rank > m || p->rank > kMaxRank)
    return fail(FINGER_EINVAL, "rank = %d out of range [0, min(m, %d)]", p->rank, kMaxRank);
  if (p->code_type < FINGER_CODE_F32 || p->code_type > FINGER_CODE_FP8E4M3)
    return fail(FINGER_EINVAL, "unknown code_type %d", p->code_type);
  if (p->metric != FINGER_L2 && p->metric != FINGER_ANGULAR && p->metric != FINGER_IP)
    return fail(FINGER_EINVAL, "unknown metric %d", p->metric);
  if (p->sigma_mode != FINGER_SIGMA_STD && p->sigma_mode != FINGER_SIGMA_VARIANCE)
    return fail(FINGER_EINVAL, "unknown sigma_mode %d", p->sigma_mode);
  if (p->n_pivots < 0 || p->n_pivots > 65536) return fail(FINGER_EINVAL, "n_pivots = %d out of range", p->n_pivots);
  if (p->n_pivots > 0 && p->pivots == nullptr) return fail(FINGER_EINVAL, "pivots is NULL with n_pivots > 0");
  if (p->dm_override && !(p->dm[3] >= 0)) return fail(FINGER_EINVAL, "dm override sigma_hat must be >= 0");
  if (p->basis != nullptr && p->rank > 0) {
    for (int64_t i = 0; i < (int64_t)p->rank * m; ++i)
      if (!std::isfinite(p->basis[i])) return fail(FINGER_EINVAL, "basis entry %lld is not finite", (long long)i);
  }
  int dev = 0;
  int st = check_device(&dev);
  if (st != FINGER_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);

  Tables* t = new (std::nothrow) Tables();
  if (t == nullptr) return fail(FINGER_ENOMEM, "host allocation failed");
  Guard guard{t};
  t->device = dev;
  t->n = n;
  t->m = m;
  t->r = p->rank;
  t->deg = max_degree;
  t->code_type = p->code_type;
  t->metric = p->metric;
  t->sigma_mode = p->sigma_mode;
  t->seed = p->seed;
  t->graph = graph;
  const int rpad = rpad_of(t->r);

  // graph and pivot checks
  DevBuf<int32_t> bad;
  if ((st = dev_alloc(reinterpret_cast<void**>(&bad.p), 8, "flags")) != FINGER_OK) return st;
  HIPCHK(hipMemsetAsync(bad.p, 0, 8, s));
  HIPCHK(launch_validate_graph(graph, n, max_degree, bad.p, s));
  if (p->n_pivots > 0) HIPCHK(launch_check_ids(p->pivots, p->n_pivots, n, bad.p + 1, s));
  int32_t hbad[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(hbad, bad.p, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hbad[0] != 0)
    return fail(FINGER_EINVAL, "graph: %d rows have an id out of range, a self loop, a repeated id or a gap before -1 padding", hbad[0]);
  if (hbad[1] != 0) return fail(FINGER_EINVAL, "pivots: %d ids out of range", hbad[1]);

  // the points the search reads
  if (t->metric == FINGER_ANGULAR) {
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->data_owned), (size_t)n * m * 4, "normalized data")) != FINGER_OK) return st;
    HIPCHK(launch_normalize_rows(data, n, m, t->data_owned, s));
    t->data = t->data_owned;
  } else {
    t->data = data;
  }
  if ((st = dev_alloc(reinterpret_cast<void**>(&t->cc), (size_t)n * 4, "node norms")) != FINGER_OK) return st;
  HIPCHK(launch_row_norms(t->data, n, m, t->cc, s));

  if (t->r > 0) {
    // ---- Algorithm 2: samples, residuals, basis, distribution matching
    const int64_t ns_req = p->n_samples > 0 ? std::min<int64_t>(p->n_samples, n)
                                            : std::min<int64_t>(n, kDefaultSamples);
    DevBuf<int32_t> raw;
    if ((st = dev_alloc(reinterpret_cast<void**>(&raw.p), (size_t)ns_req * 12, "samples")) != FINGER_OK) return st;
    HIPCHK(launch_sample_pairs(graph, n, max_degree, ns_req, p->seed, raw.p, s));
    std::vector<int32_t> hs((size_t)ns_req * 3);
    HIPCHK(hipMemcpyAsync(hs.data(), raw.p, hs.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int32_t> kept;
    kept.reserve(hs.size());
    for (int64_t i = 0; i < ns_req; ++i)
      if (hs[3 * i] >= 0) kept.insert(kept.end(), {hs[3 * i], hs[3 * i + 1], hs[3 * i + 2]});
    const int64_t ns = (int64_t)kept.size() / 3;
    if (ns < 2) return fail(FINGER_EINVAL, "fewer than 2 usable samples (nodes need >= 2 neighbours)");
    t->nsamp = ns;
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->samples), kept.size() * 4, "samples")) != FINGER_OK) return st;
    HIPCHK(hipMemcpyAsync(t->samples, kept.data(), kept.size() * 4, hipMemcpyHostToDevice, s));
    DevBuf<double> res;
    if ((st = dev_alloc(reinterpret_cast<void**>(&res.p), (size_t)ns * m * 16, "residuals")) != FINGER_OK) return st;
    double* res1 = res.p;
    double* res2 = res.p + (size_t)ns * m;
    HIPCHK(launch_residuals_f64(t->data, m, t->samples, ns, res1, res2, s));
    t->eig_host = static_cast<double*>(std::malloc((size_t)m * 8));
    t->P64_host = static_cast<double*>(std::malloc((size_t)t->r * m * 8));
    if (!t->eig_host || !t->P64_host) return fail(FINGER_ENOMEM, "host allocation failed");
    if (p->basis != nullptr) {
      // a caller-supplied basis replaces Proposition 3.1's
      std::memcpy(t->P64_host, p->basis, (size_t)t->r * m * 8);
      for (int i = 0; i < m; ++i) t->eig_host[i] = std::nan("");
    } else {
      const int parts = gram_parts(ns, m);
      DevBuf<double> gram;
      if ((st = dev_alloc(reinterpret_cast<void**>(&gram.p), (size_t)(parts + 1) * m * m * 8, "gram")) != FINGER_OK) return st;
      HIPCHK(launch_gram_f64(res1, ns, m, gram.p, s));
      std::vector<double> M((size_t)m * m);
      HIPCHK(hipMemcpyAsync(M.data(), gram.p, M.size() * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::vector<double> V((size_t)m * m);
      eigh_jacobi(M.data(), m, t->eig_host, V.data());
      std::memcpy(t->P64_host, V.data(), (size_t)t->r * m * 8);
    }
    DevBuf<double> P64d;
    if ((st = dev_alloc(reinterpret_cast<void**>(&P64d.p), (size_t)t->r * m * 8, "basis")) != FINGER_OK) return st;
    HIPCHK(hipMemcpyAsync(P64d.p, t->P64_host, (size_t)t->r * m * 8, hipMemcpyHostToDevice, s));
    // P in float, rows padded to rpad with zeros
    std::vector<float> P32((size_t)rpad * m, 0.f);
    for (int i = 0; i < t->r; ++i)
      for (int k = 0; k < m; ++k) P32[(size_t)i * m + k] = (float)t->P64_host[(size_t)i * m + k];
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->P), P32.size() * 4, "basis")) != FINGER_OK) return st;
    HIPCHK(hipMemcpyAsync(t->P, P32.data(), P32.size() * 4, hipMemcpyHostToDevice, s));
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->xy), (size_t)ns * 16, "cosines")) != FINGER_OK) return st;
    HIPCHK(launch_pair_cosines(res1, res2, ns, m, P64d.p, t->r, t->xy, s));
    DevBuf<double> sums;
    if ((st = dev_alloc(reinterpret_cast<void**>(&sums.p), 6 * 8, "sums")) != FINGER_OK) return st;
    double hsum[6];
    HIPCHK(launch_dm_sums(t->xy, ns, 0, 0, 0, 0, sums.p, s));
    HIPCHK(hipMemcpyAsync(hsum, sums.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double mu = hsum[0] / ns, mu_hat = hsum[1] / ns;
    HIPCHK(launch_dm_sums(t->xy, ns, mu, mu_hat, 0, 1, sums.p, s));
    HIPCHK(hipMemcpyAsync(hsum, sums.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double var = hsum[0] / ns, var_hat = hsum[1] / ns;
    double sigma, sigma_hat;
    if (t->sigma_mode == FINGER_SIGMA_STD) {
      sigma = std::sqrt(var);
      sigma_hat = std::sqrt(var_hat);
    } else {
      sigma = var;
      sigma_hat = var_hat;
    }
    const double scale = sigma_hat > 0 ? sigma / sigma_hat : 1.0;
    HIPCHK(launch_dm_sums(t->xy, ns, mu, mu_hat, scale, 2, sums.p, s));
    HIPCHK(hipMemcpyAsync(hsum, sums.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    t->mu = mu;
    t->sigma = sigma;
    t->mu_hat = mu_hat;
    t->sigma_hat = sigma_hat;
    t->eps = hsum[0] / ns;
    // Pearson correlation of X and Y (the rank-selection rule of Supplementary E)
    HIPCHK(launch_dm_sums(t->xy, ns, mu, mu_hat, 0, 3, sums.p, s));
    HIPCHK(hipMemcpyAsync(hsum, sums.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    t->corr_xy = (var > 0 && var_hat > 0) ? (hsum[0] / ns) / std::sqrt(var * var_hat) : 0.0;
    if (p->dm_override) {
      t->mu = p->dm[0];
      t->sigma = p->dm[1];
      t->mu_hat = p->dm[2];
      t->sigma_hat = p->dm[3];
      t->eps = p->dm[4];
    }
    // ---- node table (Supplementary G): P c for every node
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->pc), (size_t)n * rpad * 4, "node table")) != FINGER_OK) return st;
    HIPCHK(launch_gemm_nt(t->data, n, t->P, rpad, m, t->pc, rpad, s));
    // ---- edge table: alpha, rho, u per slot
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->alpha), (size_t)n * max_degree * 4, "edge alpha")) != FINGER_OK) return st;
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->rho), (size_t)n * max_degree * 4, "edge rho")) != FINGER_OK) return st;
    const size_t esz = t->code_type == FINGER_CODE_F32 ? 4 : (t->code_type == FINGER_CODE_BF16 ? 2 : 1);
    t->code_bytes = (size_t)n * max_degree * rpad * esz;
    if ((st = dev_alloc(&t->codes, t->code_bytes, "edge codes")) != FINGER_OK) return st;
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->scale), (size_t)n * 4, "code scales")) != FINGER_OK) return st;
    HIPCHK(launch_edge_codes(*t, s));
  }

  // ---- query-prep operand: P rows (padded to whole 64-column tiles), then pivots
  t->npiv = p->n_pivots;
  const int rcols = (rpad + 63) / 64 * 64;
  const int cols = rcols + (t->npiv + 63) / 64 * 64;
  t->qprep_cols = cols;
  if (cols > 0) {
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->qprep_B), (size_t)cols * m * 4, "query-prep operand")) != FINGER_OK) return st;
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->qprep_Bnorm), (size_t)cols * 4, "query-prep norms")) != FINGER_OK) return st;
    HIPCHK(hipMemsetAsync(t->qprep_B, 0, (size_t)cols * m * 4, s));
    if (t->r > 0) HIPCHK(hipMemcpyAsync(t->qprep_B, t->P, (size_t)rpad * m * 4, hipMemcpyDeviceToDevice, s));
    if (t->npiv > 0) {
      if ((st = dev_alloc(reinterpret_cast<void**>(&t->piv_ids), (size_t)t->npiv * 4, "pivots")) != FINGER_OK) return st;
      HIPCHK(hipMemcpyAsync(t->piv_ids, p->pivots, (size_t)t->npiv * 4, hipMemcpyDeviceToDevice, s));
      HIPCHK(launch_gather_rows(t->data, m, t->piv_ids, t->npiv, t->qprep_B + (size_t)rcols * m, s));
      if ((st = dev_alloc(reinterpret_cast<void**>(&t->piv_b16),
                          (size_t)pivot_pad_rows(t->npiv) * pivot_kpad(m) * 2, "bf16 pivots")) != FINGER_OK)
        return st;
      HIPCHK(launch_pack_pivots(t->qprep_B + (size_t)rcols * m, t->npiv, m, t->piv_b16, s));
    }
    HIPCHK(launch_row_norms(t->qprep_B, cols, m, t->qprep_Bnorm, s));
    if (t->npiv > 0) {
      const size_t np = (size_t)pivot_pad_rows(t->npiv);
      if ((st = dev_alloc(reinterpret_cast<void**>(&t->piv_norm), np * 4, "pivot norms")) != FINGER_OK) return st;
      HIPCHK(hipMemsetAsync(t->piv_norm, 0, np * 4, s));
      // pivot scores |p|^2 - 2 q.p rank by L2; with zero norms, -2 q.p ranks
      // by inner product
      if (t->metric != FINGER_IP)
        HIPCHK(hipMemcpyAsync(t->piv_norm, t->qprep_Bnorm + rcols, (size_t)t->npiv * 4,
                              hipMemcpyDeviceToDevice, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  guard.t = nullptr;
  *out = reinterpret_cast<finger_tables*>(t);
  return ok();
}

void finger_free_tables(finger_tables* t) { free_tables(reinterpret_cast<Tables*>(t)); }

int finger_tables_info_get(const finger_tables* th, finger_tables_info* info) {
  if (th == nullptr || info == nullptr) return fail(FINGER_EINVAL, "NULL argument");
  const Tables* t = reinterpret_cast<const Tables*>(th);
  std::memset(info, 0, sizeof(*info));
  info->n = t->n;
  info->m = t->m;
  info->rank = t->r;
  info->max_degree = t->deg;
  info->code_type = t->code_type;
  info->metric = t->metric;
  info->n_pivots = t->npiv;
  info->n_samples_used = t->nsamp;
  info->mu = t->mu;
  info->sigma = t->sigma;
  info->mu_hat = t->mu_hat;
  info->sigma_hat = t->sigma_hat;
  info->eps = t->eps;
  info->eps_gate = t->eps_gate;
  info->gate_attached = t->gate;
  info->edge_table_bytes = t->r > 0 ? (int64_t)(t->code_bytes + (size_t)t->n * t->deg * 8) : 0;
  info->corr_xy = t->corr_xy;
  info->hierarchy_top_level = t->h_top >= 0 ? t->h_top_level : 0;
  info->hierarchy_top = t->h_top;
  info->hierarchy_rows = t->h_rows;
  return ok();
}

int finger_tables_read(const finger_tables* th, int32_t which, void* dst, size_t* bytes) {
  if (th == nullptr || bytes == nullptr) return fail(FINGER_EINVAL, "NULL argument");
  const Tables* t = reinterpret_cast<const Tables*>(th);
  const int rpad = rpad_of(t->r);
  const void* src = nullptr;
  size_t sz = 0;
  bool host = false;
  bool strip = false;  // rows of rpad floats copied as rows of r
  int64_t rows = 0;
  switch (which) {
    case FINGER_T_P_F64: src = t->P64_host; sz = (size_t)t->r * t->m * 8; host = true; break;
    case FINGER_T_EIGVALS: src = t->eig_host; sz = t->r > 0 ? (size_t)t->m * 8 : 0; host = true; break;
    case FINGER_T_P_F32: src = t->P; sz = (size_t)t->r * t->m * 4; break;
    case FINGER_T_NODE_CC: src = t->cc; sz = (size_t)t->n * 4; break;
    case FINGER_T_NODE_PC: src = t->pc; sz = (size_t)t->n * t->r * 4; strip = true; rows = t->n; break;
    case FINGER_T_EDGE_ALPHA: src = t->alpha; sz = t->r > 0 ? (size_t)t->n * t->deg * 4 : 0; break;
    case FINGER_T_EDGE_RHO: src = t->rho; sz = t->r > 0 ? (size_t)t->n * t->deg * 4 : 0; break;
    case FINGER_T_EDGE_CODES: src = t->codes; sz = t->code_bytes; break;
    case FINGER_T_EDGE_SCALE: src = t->scale; sz = t->r > 0 ? (size_t)t->n * 4 : 0; break;
    case FINGER_T_SAMPLES: src = t->samples; sz = (size_t)t->nsamp * 12; break;
    case FINGER_T_XY: src = t->xy; sz = (size_t)t->nsamp * 16; break;
    default: return fail(FINGER_EINVAL, "unknown table selector %d", which);
  }
  if (dst == nullptr) {
    *bytes = sz;
    return ok();
  }
  if (*bytes < sz) {
    const size_t cap = *bytes;
    *bytes = sz;
    return fail(FINGER_EOVERFLOW, "table needs %zu bytes, buffer has %zu", sz, cap);
  }
  *bytes = sz;
  if (sz == 0) return ok();
  if (host) {
    std::memcpy(dst, src, sz);
  } else if (strip && rpad != t->r) {
    HIPCHK(hipMemcpy2D(dst, (size_t)t->r * 4, src, (size_t)rpad * 4, (size_t)t->r * 4, (size_t)rows,
                       hipMemcpyDeviceToHost));
  } else {
    HIPCHK(hipMemcpy(dst, src, sz, hipMemcpyDeviceToHost));
  }
  return ok();
}

}  // extern "C"

// ----------------------------------------------------------------- search

namespace {

struct Plan {
  int ef_max, vis_cap, waves, lds, spill_slots;
  size_t off_qq, off_pq, off_ent, off_queue, off_qscr, off_spill, off_qn, total;
  // ef classes (a partitioned search with per-query K/ef): one launch per
  // class, each sized for its own bound
  finger::ClassBounds cb;
  int cls_vis[finger::kMaxEfClasses], cls_waves[finger::kMaxEfClasses], cls_spill[finger::kMaxEfClasses];
  size_t off_lists, off_counts;
};

int plan_search(const Tables* t, int64_t nq, const finger_search_params* p, Plan* pl) {
  using namespace finger;
  if (p->mode < FINGER_MODE_PLAIN || p->mode > FINGER_MODE_GATED)
    return fail(FINGER_EINVAL, "unknown mode %d", p->mode);
  if (p->mode != FINGER_MODE_PLAIN && t->r == 0)
    return fail(FINGER_EINVAL, "FINGER modes need a handle built with rank > 0");
  if (t->metric == FINGER_IP && (p->mode == FINGER_MODE_GATED || p->log_features != nullptr))
    return fail(FINGER_EINVAL, "the learned gate and its feature log are for L2 and angular only");
  if (p->mode == FINGER_MODE_GATED && !t->gate)
    return fail(FINGER_EINVAL, "gated mode needs finger_gate_attach first");
  if (nq < 0) return fail(FINGER_EINVAL, "nq < 0");
  const bool perq = p->k_per_query != nullptr || p->ef_per_query != nullptr;
  if (p->k_per_query == nullptr && (p->k < 1 || p->k > t->n))
    return fail(FINGER_EINVAL, "k = %d out of range [1, n]", p->k);
  if (p->ef_per_query == nullptr && p->ef < 1) return fail(FINGER_EINVAL, "ef = %d < 1", p->ef);
  const int kmax_needed = p->k_per_query == nullptr ? p->k : 1;
  if (p->k_max < kmax_needed) return fail(FINGER_EINVAL, "k_max = %d < k = %d", p->k_max, p->k);
  if (p->entry < FINGER_ENTRY_DESCENT || p->entry >= t->n)
    return fail(FINGER_EINVAL, "entry = %d out of range", p->entry);
  if (p->entry == FINGER_ENTRY_PIVOT && t->npiv == 0)
    return fail(FINGER_EINVAL, "entry = -1 needs pivots in the tables");
  if (p->entry == FINGER_ENTRY_DESCENT && t->h_top < 0)
    return fail(FINGER_EINVAL, "entry = -2 needs upper layers (finger_hierarchy_attach)");
  int ef_max = p->ef_max;
  if (perq) {
    if (ef_max < 1) return fail(FINGER_EINVAL, "ef_max must be set with per-query k or ef");
  } else {
    const int need = std::max(p->ef, p->k);
    if (ef_max < need) ef_max = need;
  }
  if (ef_max > kMaxEf) return fail(FINGER_EOVERFLOW, "ef_max = %d exceeds %d", ef_max, kMaxEf);
  if (p->ef_classes < 0 || p->ef_classes > 3)
    return fail(FINGER_EINVAL, "ef_classes = %d must be 0, 1, 2 or 3", p->ef_classes);
  // visited-set slots in LDS: 2048 (8 KB) for every ef.  A query visits about
  // as many nodes as it computes distances for, and measured on the 1M- and
  // 10M-point workloads up to ef = 512 a 2048-slot table (spilling to the
  // global table beyond) beats larger ones, which cost resident waves
  auto vis_default = [](int) { return 2048; };
  int vis_cap = p->visited_capacity;
  if (vis_cap == 0) vis_cap = vis_default(ef_max);
  if (p->code_prefetch < -1 || p->code_prefetch > 1)
    return fail(FINGER_EINVAL, "code_prefetch = %d must be -1, 0 or 1", p->code_prefetch);
  if (!(p->gate_band >= 0.f) || p->gate_band > 1e30f)
    return fail(FINGER_EINVAL, "gate_band must be a finite value >= 0");
  if (p->screen_layout < 0 || p->screen_layout > 2)
    return fail(FINGER_EINVAL, "screen_layout = %d must be 0, 1 or 2", p->screen_layout);
  if (vis_cap < 256 || (vis_cap & (vis_cap - 1)) != 0)
    return fail(FINGER_EINVAL, "visited_capacity = %d must be a power of two >= 256", vis_cap);
  if (p->visited_probe != 0 && (p->visited_probe < 4 || p->visited_probe > 64 || (p->visited_probe & 3) != 0))
    return fail(FINGER_EINVAL, "visited_probe = %d must be 0 or a multiple of 4 in [4, 64]", p->visited_probe);
  const int gate_in = p->mode == FINGER_MODE_GATED ? t->gate_in : 0;
  const int r_used = p->mode == FINGER_MODE_PLAIN ? 0 : t->r;
  const int lds_wave = search_lds_bytes(ef_max, vis_cap, r_used, t->m, gate_in);
  const int lds_shared = 0;
  const int lds_limit = 160 * 1024;
  const int wpb = 1;
  if (lds_shared + wpb * lds_wave > lds_limit)
    return fail(FINGER_EOVERFLOW, "per-wave LDS of %d bytes (ef_max %d, visited %d) exceeds the CU budget", lds_wave, ef_max, vis_cap);
  int per_cu = p->waves_per_cu;
  const int lds_fit = (lds_limit / (lds_shared + wpb * lds_wave)) * wpb;
  if (per_cu <= 0) per_cu = std::min(16, lds_fit);
  if (per_cu > 32) return fail(FINGER_EINVAL, "waves_per_cu = %d > 32", per_cu);
  per_cu = std::min(per_cu, lds_fit);
  int waves = per_cu * cu_count();
  if (nq < waves) waves = (int)std::max<int64_t>(nq, 1);
  waves = (waves + wpb - 1) / wpb * wpb;
  const int rpad = rpad_of(t->r);
  size_t off = 0;
  pl->off_qq = off;  off += align256((size_t)nq * 4);
  pl->off_pq = off;  off += align256((size_t)nq * rpad * 4);
  pl->off_ent = off; off += align256((size_t)nq * 4);
  pl->off_queue = off; off += 256;
  pl->off_qscr = off; off += align256(query_prep_scratch_bytes(*t, nq));
  auto spill_default = [&](int ef) { return std::min(65536, std::max(1024, next_pow2(ef * t->deg))); };
  int spill_slots = p->spill_capacity;
  if (spill_slots == 0) spill_slots = spill_default(ef_max);
  if (spill_slots < 64 || spill_slots > (1 << 20) || (spill_slots & (spill_slots - 1)) != 0)
    return fail(FINGER_EINVAL, "spill_capacity = %d must be a power of two in [64, 2^20]", spill_slots);
  // ef classes: bounds 32, 64, ... below ef_max, then ef_max
  pl->cb.n = 0;
  size_t spill_words = (size_t)waves * spill_slots;
  if (perq && p->ef_classes != 2) {
    for (int b = 32; b < ef_max && pl->cb.n < kMaxEfClasses - 1; b *= 2) pl->cb.bound[pl->cb.n++] = b;
    pl->cb.bound[pl->cb.n++] = ef_max;
    for (int c = 0; c < pl->cb.n; ++c) {
      const int b = pl->cb.bound[c];
      const int vc = p->visited_capacity ? p->visited_capacity : vis_default(b);
      const int lw = search_lds_bytes(b, vc, r_used, t->m, gate_in);
      if (lw > lds_limit) return fail(FINGER_EOVERFLOW, "per-wave LDS of %d bytes for ef class %d exceeds the CU budget", lw, b);
      const int fit = lds_limit / lw;
      int pc = p->waves_per_cu > 0 ? std::min(p->waves_per_cu, fit) : std::min(16, fit);
      int wv = pc * cu_count();
      if (nq < wv) wv = (int)std::max<int64_t>(nq, 1);
      pl->cls_vis[c] = vc;
      pl->cls_waves[c] = wv;
      pl->cls_spill[c] = p->spill_capacity ? p->spill_capacity : spill_default(b);
      spill_words = std::max(spill_words, (size_t)wv * pl->cls_spill[c]);
    }
  }
  pl->off_spill = off; off += align256(spill_words * 4);
  pl->off_lists = off;
  if (pl->cb.n > 0) off += align256((size_t)pl->cb.n * nq * 4);
  pl->off_counts = off;
  if (pl->cb.n > 0) off += 256;
  pl->spill_slots = spill_slots;
  // angular metric: the search reads unit-normalized copies of the queries
  pl->off_qn = off;
  if (t->metric == FINGER_ANGULAR) off += align256((size_t)nq * t->m * 4);
  pl->total = off;
  pl->ef_max = ef_max;
  pl->vis_cap = vis_cap;
  pl->waves = waves;
  pl->lds = lds_wave;
  return FINGER_OK;
}

}  // namespace

extern "C" {

int finger_search_workspace_size(const finger_tables* th, int64_t nq, const finger_search_params* p,
                                 size_t* bytes) {
  if (th == nullptr || p == nullptr || bytes == nullptr) return fail(FINGER_EINVAL, "NULL argument");
  Plan pl;
  int st = plan_search(reinterpret_cast<const Tables*>(th), nq, p, &pl);
  if (st != FINGER_OK) return st;
  *bytes = pl.total;
  return ok();
}

int finger_search(const finger_tables* th, const float* queries, int64_t nq,
                  const finger_search_params* p, int32_t* out_ids, float* out_dist,
                  int32_t* out_counters, void* workspace, size_t workspace_bytes, void* stream) {
  using namespace finger;
  if (th == nullptr || p == nullptr) return fail(FINGER_EINVAL, "NULL handle or params");
  const Tables* t = reinterpret_cast<const Tables*>(th);
  Plan pl;
  int st = plan_search(t, nq, p, &pl);
  if (st != FINGER_OK) return st;
  if (nq == 0) return ok();
  if (queries == nullptr || out_ids == nullptr || out_dist == nullptr)
    return fail(FINGER_EINVAL, "queries/out_ids/out_dist is NULL");
  if ((reinterpret_cast<uintptr_t>(queries) & 15u) != 0) return fail(FINGER_EINVAL, "queries must be 16-byte aligned");
  if (workspace == nullptr || workspace_bytes < pl.total)
    return fail(FINGER_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, pl.total);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(FINGER_EINVAL, "workspace must be 256-byte aligned");
  if (p->log_features != nullptr && (p->mode != FINGER_MODE_FINGER || p->log_targets == nullptr || p->log_count == nullptr))
    return fail(FINGER_EINVAL, "feature logging needs mode FINGER, log_targets and log_count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float* qq = reinterpret_cast<float*>(ws + pl.off_qq);
  float* pq = reinterpret_cast<float*>(ws + pl.off_pq);
  int32_t* ent = reinterpret_cast<int32_t*>(ws + pl.off_ent);
  int32_t* queue = reinterpret_cast<int32_t*>(ws + pl.off_queue);  // [kMaxEfClasses]
  float* qscr = reinterpret_cast<float*>(ws + pl.off_qscr);
  int32_t* spill = reinterpret_cast<int32_t*>(ws + pl.off_spill);
  if (t->metric == FINGER_ANGULAR) {
    float* qn = reinterpret_cast<float*>(ws + pl.off_qn);
    HIPCHK(launch_normalize_rows(queries, nq, t->m, qn, s));
    queries = qn;
  }
  // a fill kernel rather than a memset: a caller may capture this call in a
  // graph.  The visited-set spill tables need no fill: each wave empties its
  // own the first time it needs it.
  HIPCHK(launch_fill_u32(queue, 0u, kMaxEfClasses, s));
  const bool need_prep = p->mode != FINGER_MODE_PLAIN || p->entry == FINGER_ENTRY_PIVOT;
  if (need_prep)
    HIPCHK(launch_query_prep(*t, queries, nq, qq, pq, p->entry == FINGER_ENTRY_PIVOT ? ent : nullptr,
                             qscr, s, p->mode != FINGER_MODE_PLAIN));
  if (p->entry == FINGER_ENTRY_DESCENT) HIPCHK(launch_descend(*t, queries, nq, ent, nullptr, s));
  SearchLaunch L{};
  L.queries = queries;
  L.nq = nq;
  L.mode = p->mode;
  L.k_all = p->k;
  L.ef_all = p->ef;
  L.k_max = p->k_max;
  L.ef_max = pl.ef_max;
  L.entry = p->entry;
  L.warmup = p->warmup < 0 ? 5 : p->warmup;
  L.kq = p->k_per_query;
  L.efq = p->ef_per_query;
  L.qq = qq;
  L.pq = pq;
  L.entries = p->entry < 0 ? ent : nullptr;
  L.out_ids = out_ids;
  L.out_dist = out_dist;
  L.counters = out_counters;
  L.queue = queue;
  L.spill = spill;
  L.spill_slots_per_wave = pl.spill_slots;
  L.vis_cap = pl.vis_cap;
  L.vis_probe = p->visited_probe ? p->visited_probe : 24;
  L.waves = pl.waves;
  L.persistent = p->persistent;
  L.prefetch = p->code_prefetch > 0;
  L.coalesced = p->screen_layout != 2;
  L.gate_band = p->gate_band;
  L.log_x = p->log_features;
  L.log_y = p->log_targets;
  L.log_cap = p->log_capacity;
  L.log_count = p->log_count;
  hipEvent_t ev0 = static_cast<hipEvent_t>(p->kernel_events[0]);
  hipEvent_t ev1 = static_cast<hipEvent_t>(p->kernel_events[1]);
  int32_t* lists = reinterpret_cast<int32_t*>(ws + pl.off_lists);
  int32_t* counts = reinterpret_cast<int32_t*>(ws + pl.off_counts);
  if (pl.cb.n > 0) HIPCHK(launch_ef_classes(p->k_per_query, p->ef_per_query, nq, p->k, p->ef, pl.cb, counts, lists, s));
  if (ev0) HIPCHK(hipEventRecord(ev0, s));
  if (pl.cb.n == 0) {
    HIPCHK(launch_search(*t, L, s));
  } else if (p->ef_classes == 0 || p->ef_classes == 3) {
    // one persistent launch reserving for ef_max, its queue serving the
    // largest ef class first (the short queries fill the launch's end)
    SearchLaunch Lc = L;
    Lc.persistent = 1;
    Lc.qlist = lists;
    Lc.qcount = counts;
    Lc.nclass = pl.cb.n;
    Lc.list_stride = nq;
    HIPCHK(launch_search(*t, Lc, s));
  } else {
    // one persistent launch per ef class, each sized for its own bound
    for (int c = 0; c < pl.cb.n; ++c) {
      SearchLaunch Lc = L;
      Lc.ef_max = pl.cb.bound[c];
      Lc.vis_cap = pl.cls_vis[c];
      Lc.waves = pl.cls_waves[c];
      Lc.spill_slots_per_wave = pl.cls_spill[c];
      Lc.persistent = 1;
      Lc.queue = queue + c;
      Lc.qlist = lists + (int64_t)c * nq;
      Lc.qcount = counts + c;
      HIPCHK(launch_search(*t, Lc, s));
    }
  }
  if (ev1) HIPCHK(hipEventRecord(ev1, s));
  return ok();
}

}  // extern "C"

// ------------------------------------------------ search without allocation

namespace {

// Scratch of finger_search_noalloc: a fixed array in the code object's
// device memory, one copy per GPU, held until the process ends.  In host
// code the name only stands in for the array; its address on a device comes
// from hipGetSymbolAddress (once per device, with that device current) and
// is the only form passed to kernels or fills.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FINGER_EDEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(FINGER_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return FINGER_OK;
}

}  // namespace

extern "C" {

size_t finger_search_noalloc_capacity(void) { return kNoAllocScratchBytes; }

int finger_search_noalloc(const finger_tables* th, const float* queries, int64_t nq,
                          const finger_search_params* p, int32_t* out_ids, float* out_dist,
                          int32_t* out_counters, void* stream) {
  if (th == nullptr || p == nullptr) return fail(FINGER_EINVAL, "NULL handle or params");
  Plan pl;
  const int st = plan_search(reinterpret_cast<const Tables*>(th), nq, p, &pl);
  if (st != FINGER_OK) return st;
  if (pl.total > kNoAllocScratchBytes)
    return fail(FINGER_EOVERFLOW,
                "the search needs %zu bytes of scratch, more than the %zu finger_search_noalloc holds "
                "(fewer queries per call, or finger_search with a workspace)",
                pl.total, kNoAllocScratchBytes);
  void* ws = nullptr;
  const int sa = scratch_address(&ws);
  if (sa != FINGER_OK) return sa;
  return finger_search(th, queries, nq, p, out_ids, out_dist, out_counters, ws, kNoAllocScratchBytes,
                       stream);
}

}  // extern "C"

namespace {

// The graph recipe of finger_build_graph; with groups (host offsets
// group[0] = 0 < ... < group[n_groups] = n) each point's kNN is taken among
// the points of its own group only.
int build_graph_impl(const float* data, int64_t n, int32_t m, int32_t knn_k, int32_t max_degree,
                     int32_t metric, int32_t entry, const int64_t* groups, int64_t n_groups,
                     int32_t* out_graph, finger_graph_stats* stats, finger_progress_fn progress,
                     void* progress_user, void* stream) {
  using namespace finger;
  if (data == nullptr || out_graph == nullptr) return fail(FINGER_EINVAL, "NULL data or out_graph");
  if (n < 2) return fail(FINGER_EINVAL, "n = %lld < 2", (long long)n);
  if (m <= 0 || m > kMaxDim || m % 4 != 0) return fail(FINGER_EINVAL, "m = %d must be a multiple of 4 in [4, %d]", m, kMaxDim);
  if (knn_k < 1 || knn_k > 127 || knn_k > n - 1)
    return fail(FINGER_EINVAL, "knn_k = %d out of range [1, min(n - 1, 127)]", knn_k);
  if (max_degree < 1 || max_degree > kMaxDegree)
    return fail(FINGER_EINVAL, "max_degree = %d out of range [1, %d]", max_degree, kMaxDegree);
  if (metric != FINGER_L2 && metric != FINGER_ANGULAR)
    return fail(FINGER_EINVAL, "metric %d: the graph recipe needs L2 or angular distances", metric);
  if (entry < 0 || entry >= n) return fail(FINGER_EINVAL, "entry = %d out of range", entry);
  if ((reinterpret_cast<uintptr_t>(data) & 15u) != 0) return fail(FINGER_EINVAL, "data must be 16-byte aligned");
  const int k = knn_k, k1 = knn_k + 1, W = max_degree;
  const int64_t nk = n * k, ne = 2 * nk;
  int64_t gmax = 0;
  if (groups != nullptr) {
    if (n_groups < 1 || groups[0] != 0 || groups[n_groups] != n)
      return fail(FINGER_EINVAL, "group offsets must run from 0 to n");
    for (int64_t g = 0; g < n_groups; ++g) {
      const int64_t sz = groups[g + 1] - groups[g];
      if (sz < k1) return fail(FINGER_EINVAL, "group %lld holds %lld points, fewer than knn_k + 1", (long long)g, (long long)sz);
      gmax = std::max(gmax, sz);
    }
  }
  if (ne >= (int64_t(1) << 31)) return fail(FINGER_EOVERFLOW, "2 n knn_k = %lld >= 2^31", (long long)ne);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms_since = [&](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(now() - t0).count();
  };
  finger_graph_stats st{};
  int rc = FINGER_OK;
  auto alloc = [&](auto& buf, size_t bytes, const char* what) {
    if (rc == FINGER_OK) rc = dev_alloc(reinterpret_cast<void**>(&buf.p), std::max<size_t>(bytes, 4), what);
  };

  // 1. kNN (k + 1 with the point itself, which is then dropped)
  auto t0 = now();
  DevBuf<float> normed;
  const float* X = data;
  if (metric == FINGER_ANGULAR) {
    alloc(normed, (size_t)n * m * 4, "normalized points");
    if (rc != FINGER_OK) return rc;
    HIPCHK(launch_normalize_rows(data, n, m, normed.p, s));
    X = normed.p;
  }
  const int64_t batch = groups != nullptr ? std::min<int64_t>(gmax, int64_t(1) << 20)
                                          : std::min<int64_t>(n, int64_t(1) << 20);
  DevBuf<char> kws;
  DevBuf<int32_t> ids1, ids;
  DevBuf<float> d1, dk;
  alloc(kws, exact_knn_ws_bytes(groups != nullptr ? gmax : n, m, batch, k1), "kNN workspace");
  alloc(ids1, (size_t)batch * k1 * 4, "kNN ids");
  alloc(d1, (size_t)batch * k1 * 4, "kNN distances");
  alloc(ids, (size_t)nk * 4, "kNN lists");
  alloc(dk, (size_t)nk * 4, "kNN list distances");
  if (rc != FINGER_OK) return rc;
  if (groups == nullptr) {
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
      const int64_t nb = std::min(batch, n - b0);
      HIPCHK(launch_exact_knn(X, n, m, X + b0 * m, nb, k1, FINGER_L2, ids1.p, d1.p, kws.p, s));
      HIPCHK(launch_drop_self(ids1.p, d1.p, nb, k1, k, ids.p + b0 * k, dk.p + b0 * k, b0, 0, s));
      HIPCHK(hipStreamSynchronize(s));
      if (progress) progress("knn", b0 + nb, n, progress_user);
    }
  } else {
    for (int64_t g = 0; g < n_groups; ++g) {
      const int64_t o = groups[g], ng = groups[g + 1] - groups[g];
      for (int64_t b0 = 0; b0 < ng; b0 += batch) {
        const int64_t nb = std::min(batch, ng - b0);
        HIPCHK(launch_exact_knn(X + o * m, ng, m, X + (o + b0) * m, nb, k1, FINGER_L2, ids1.p, d1.p, kws.p, s));
        HIPCHK(launch_drop_self(ids1.p, d1.p, nb, k1, k, ids.p + (o + b0) * k, dk.p + (o + b0) * k, b0, o, s));
      }
      if ((g + 1) % 1024 == 0 || g + 1 == n_groups) {
        HIPCHK(hipStreamSynchronize(s));
        if (progress) progress("knn", groups[g + 1], n, progress_user);
      }
    }
  }
  st.ms_knn = ms_since(t0);
  kws.reset();
  ids1.reset();
  d1.reset();

  // 2. symmetrization: stable sorts by target, then by (source, distance)
  t0 = now();
  int nbits = 1;
  while ((int64_t(1) << nbits) < n) ++nbits;
  DevBuf<uint32_t> ka, kb, va, vb, cnt, indptr;
  DevBuf<uint64_t> k2a, k2b;
  DevBuf<char> tmp;
  alloc(ka, (size_t)ne * 4, "edge keys");
  alloc(kb, (size_t)ne * 4, "edge keys");
  alloc(va, (size_t)ne * 4, "edge order");
  alloc(vb, (size_t)ne * 4, "edge order");
  alloc(k2a, (size_t)ne * 8, "edge keys");
  alloc(k2b, (size_t)ne * 8, "edge keys");
  alloc(cnt, (size_t)(n + 1) * 4, "row counts");
  alloc(indptr, (size_t)(n + 1) * 4, "row offsets");
  if (rc != FINGER_OK) return rc;
  size_t tb1 = 0, tb2 = 0, tb3 = 0, tb4 = 0;
  HIPCHK(radix_sort_u32(nullptr, tb1, ka.p, kb.p, va.p, vb.p, ne, nbits, s));
  HIPCHK(radix_sort_u64(nullptr, tb2, k2a.p, k2b.p, vb.p, va.p, ne, 32 + nbits, s));
  HIPCHK(exclusive_sum_u32(nullptr, tb3, ka.p, kb.p, ne, s));
  HIPCHK(exclusive_sum_u32(nullptr, tb4, cnt.p, indptr.p, n + 1, s));
  size_t tbytes = std::max(std::max(tb1, tb2), std::max(tb3, tb4));
  alloc(tmp, tbytes, "sort scratch");
  if (rc != FINGER_OK) return rc;
  HIPCHK(launch_sym_keys_dst(n, k, ids.p, dk.p, ka.p, va.p, s));
  size_t tb = tbytes;
  HIPCHK(radix_sort_u32(tmp.p, tb, ka.p, kb.p, va.p, vb.p, ne, nbits, s));
  HIPCHK(launch_sym_keys_src_d(n, k, ids.p, dk.p, vb.p, k2a.p, s));
  tb = tbytes;
  HIPCHK(radix_sort_u64(tmp.p, tb, k2a.p, k2b.p, vb.p, va.p, ne, 32 + nbits, s));
  // va: edges by (source, distance, target); ka = keep flags, kb = kept rank
  HIPCHK(launch_fill_u32(cnt.p, 0u, (size_t)(n + 1), s));
  HIPCHK(launch_sym_dedupe(n, k, ids.p, dk.p, va.p, ka.p, cnt.p, s));
  tb = tbytes;
  HIPCHK(exclusive_sum_u32(tmp.p, tb, ka.p, kb.p, ne, s));
  tb = tbytes;
  HIPCHK(exclusive_sum_u32(tmp.p, tb, cnt.p, indptr.p, n + 1, s));
  std::vector<uint32_t> ip_h;
  try {
    ip_h.resize((size_t)n + 1);
  } catch (const std::bad_alloc&) {
    return fail(FINGER_ENOMEM, "host row offsets");
  }
  HIPCHK(hipMemcpyAsync(ip_h.data(), indptr.p, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t total = ip_h[(size_t)n];
  uint32_t dmax = 0;
  for (int64_t i = 0; i < n; ++i) dmax = std::max(dmax, ip_h[(size_t)i + 1] - ip_h[(size_t)i]);
  st.sym_edges = total;
  st.sym_degree_max = (int32_t)dmax;
  DevBuf<int32_t> nbr;
  DevBuf<float> nd;
  alloc(nbr, (size_t)total * 4, "symmetrized rows");
  alloc(nd, (size_t)total * 4, "symmetrized distances");
  if (rc != FINGER_OK) return rc;
  HIPCHK(launch_sym_fill(n, k, ids.p, dk.p, va.p, ka.p, kb.p, nbr.p, nd.p, s));
  HIPCHK(hipStreamSynchronize(s));
  st.ms_symmetrize = ms_since(t0);
  if (progress) progress("symmetrize", total, total, progress_user);

  // 3. neighbour-selection heuristic on long rows
  t0 = now();
  HIPCHK(launch_prune(X, n, m, indptr.p, nbr.p, nd.p, W, out_graph, s));
  HIPCHK(hipStreamSynchronize(s));
  st.ms_prune = ms_since(t0);
  if (progress) progress("prune", n, n, progress_user);

  // 4. reachability repair from the entry (host loop; each step depends on the last)
  t0 = now();
  DevBuf<int32_t> deg, fa, fb;
  DevBuf<uint32_t> reached, ctr;
  DevBuf<unsigned long long> best;
  alloc(deg, (size_t)n * 4, "degrees");
  alloc(fa, (size_t)n * 4, "BFS frontier");
  alloc(fb, (size_t)n * 4, "BFS frontier");
  alloc(reached, (size_t)n * 4, "reached flags");
  alloc(ctr, 4, "BFS counter");
  alloc(best, 8, "nearest key");
  if (rc != FINGER_OK) return rc;
  std::vector<int32_t> deg_h, row_h((size_t)W), next_h;
  std::vector<uint8_t> reached_h;
  try {
    deg_h.resize((size_t)n);
    reached_h.assign((size_t)n, 0);
    next_h.resize((size_t)n);
  } catch (const std::bad_alloc&) {
    return fail(FINGER_ENOMEM, "host repair state");
  }
  HIPCHK(launch_degrees(out_graph, n, W, deg.p, s));
  HIPCHK(launch_fill_u32(reached.p, 0u, (size_t)n, s));
  HIPCHK(hipMemcpyAsync(deg_h.data(), deg.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto put = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
  };
  auto get = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
  };
  const uint32_t one = 1u, zero = 0u;
  auto mark_from = [&](int32_t start) -> hipError_t {
    reached_h[(size_t)start] = 1;
    hipError_t e = put(reached.p + start, &one, 4);
    if (e == hipSuccess) e = put(fa.p, &start, 4);
    int32_t* cur = fa.p;
    int32_t* nxt = fb.p;
    int64_t fsize = 1;
    while (e == hipSuccess && fsize > 0) {
      e = put(ctr.p, &zero, 4);
      if (e == hipSuccess) e = launch_bfs_level(out_graph, W, cur, fsize, reached.p, nxt, ctr.p, s);
      uint32_t got = 0;
      if (e == hipSuccess) e = get(&got, ctr.p, 4);
      if (e == hipSuccess && got > 0) e = get(next_h.data(), nxt, (size_t)got * 4);
      for (uint32_t t = 0; e == hipSuccess && t < got; ++t) reached_h[(size_t)next_h[t]] = 1;
      std::swap(cur, nxt);
      fsize = got;
    }
    return e;
  };
  HIPCHK(mark_from(entry));
  int64_t u = 0;
  int repairs = 0;
  int64_t added = 0;
  while (true) {
    while (u < n && reached_h[(size_t)u]) ++u;
    if (u == n) break;
    ++repairs;
    const unsigned long long none = ~0ull;
    HIPCHK(put(best.p, &none, 8));
    HIPCHK(launch_nearest_free(X, n, m, (int)u, reached.p, deg.p, W, best.p, s));
    unsigned long long bk = 0;
    HIPCHK(get(&bk, best.p, 8));
    if (bk == none) return fail(FINGER_EOVERFLOW, "repair of node %lld: no reached node has a free slot", (long long)u);
    const int32_t v = (int32_t)(uint32_t)bk;
    const int32_t uu = (int32_t)u;
    HIPCHK(put(out_graph + (int64_t)v * W + deg_h[(size_t)v], &uu, 4));
    ++deg_h[(size_t)v];
    HIPCHK(put(deg.p + v, &deg_h[(size_t)v], 4));
    ++added;
    if (deg_h[(size_t)u] < W) {
      HIPCHK(get(row_h.data(), out_graph + u * W, (size_t)W * 4));
      bool has = false;
      for (int t = 0; t < deg_h[(size_t)u]; ++t) has = has || row_h[(size_t)t] == v;
      if (!has) {
        HIPCHK(put(out_graph + u * W + deg_h[(size_t)u], &v, 4));
        ++deg_h[(size_t)u];
        HIPCHK(put(deg.p + u, &deg_h[(size_t)u], 4));
        ++added;
      }
    }
    HIPCHK(mark_from(uu));
  }
  st.components_before_repair = repairs + 1;
  st.edges_added = added;
  st.ms_repair = ms_since(t0);
  if (progress) progress("repair", repairs, repairs, progress_user);
  if (stats != nullptr) *stats = st;
  return ok();
}

}  // namespace

extern "C" {

int finger_build_graph(const float* data, int64_t n, int32_t m, int32_t knn_k, int32_t max_degree,
                       int32_t metric, int32_t entry, int32_t* out_graph, finger_graph_stats* stats,
                       finger_progress_fn progress, void* progress_user, void* stream) {
  return build_graph_impl(data, n, m, knn_k, max_degree, metric, entry, nullptr, 0, out_graph, stats,
                          progress, progress_user, stream);
}

int finger_build_graph_grouped(const float* data, int64_t n, int32_t m, int32_t knn_k,
                               int32_t max_degree, int32_t metric, int32_t entry,
                               const int64_t* group_offsets, int64_t n_groups, int32_t* out_graph,
                               finger_graph_stats* stats, finger_progress_fn progress,
                               void* progress_user, void* stream) {
  if (group_offsets == nullptr) return fail(FINGER_EINVAL, "group_offsets is NULL");
  return build_graph_impl(data, n, m, knn_k, max_degree, metric, entry, group_offsets, n_groups,
                          out_graph, stats, progress, progress_user, stream);
}

int finger_hierarchy_attach(finger_tables* th, const int32_t* levels, const int32_t* upper,
                            int64_t rows, int32_t width) {
  using namespace finger;
  if (th == nullptr || levels == nullptr) return fail(FINGER_EINVAL, "NULL handle or levels");
  if (rows < 0) return fail(FINGER_EINVAL, "rows = %lld < 0", (long long)rows);
  if (rows > 0 && upper == nullptr) return fail(FINGER_EINVAL, "upper is NULL with rows > 0");
  if (width < 1 || width > kMaxDegree) return fail(FINGER_EINVAL, "width = %d out of range [1, %d]", width, kMaxDegree);
  if (rows >= (int64_t(1) << 31)) return fail(FINGER_EOVERFLOW, "rows = %lld >= 2^31", (long long)rows);
  Tables* t = reinterpret_cast<Tables*>(th);
  const int64_t n = t->n;
  std::vector<int32_t> lv, up, row0;
  try {
    lv.resize((size_t)n);
    up.resize((size_t)rows * width);
    row0.resize((size_t)n);
  } catch (const std::bad_alloc&) {
    return fail(FINGER_ENOMEM, "host copy of the hierarchy (%lld rows)", (long long)rows);
  }
  HIPCHK(hipMemcpy(lv.data(), levels, (size_t)n * 4, hipMemcpyDeviceToHost));
  if (rows > 0) HIPCHK(hipMemcpy(up.data(), upper, up.size() * 4, hipMemcpyDeviceToHost));
  int64_t sum = 0;
  int top_level = 0, top = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (lv[i] < 0 || lv[i] > 64) return fail(FINGER_EINVAL, "levels[%lld] = %d out of range [0, 64]", (long long)i, lv[i]);
    row0[i] = lv[i] > 0 ? (int32_t)sum : -1;
    sum += lv[i];
    if (lv[i] > top_level) { top_level = lv[i]; top = (int)i; }
  }
  if (sum != rows) return fail(FINGER_EINVAL, "rows = %lld but the levels sum to %lld", (long long)rows, (long long)sum);
  for (int64_t i = 0; i < n; ++i)
    for (int l = 1; l <= lv[i]; ++l) {
      const int32_t* r = up.data() + (size_t)(row0[i] + l - 1) * width;
      for (int j = 0; j < width; ++j) {
        const int32_t v = r[j];
        if (v == -1) continue;
        if (v < -1 || v >= n || v == i || lv[v] < l)
          return fail(FINGER_EINVAL, "node %lld layer %d: neighbour %d is out of range, the node itself or not in the layer",
                      (long long)i, l, v);
      }
    }
  int32_t *d_row0 = nullptr, *d_up = nullptr;
  int st = dev_alloc(reinterpret_cast<void**>(&d_row0), (size_t)n * 4, "hierarchy row offsets");
  if (st != FINGER_OK) return st;
  if ((st = dev_alloc(reinterpret_cast<void**>(&d_up), std::max<size_t>(up.size() * 4, 4), "hierarchy rows")) != FINGER_OK) {
    (void)hipFree(d_row0);
    return st;
  }
  hipError_t e = hipMemcpy(d_row0, row0.data(), (size_t)n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && rows > 0) e = hipMemcpy(d_up, up.data(), up.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d_row0);
    (void)hipFree(d_up);
    return fail(FINGER_EDEVICE, "copying the hierarchy: %s", hipGetErrorString(e));
  }
  if (t->h_row0) (void)hipFree(t->h_row0);
  if (t->h_upper) (void)hipFree(t->h_upper);
  t->h_row0 = d_row0;
  t->h_upper = d_up;
  t->h_rows = rows;
  t->h_width = width;
  t->h_top_level = top_level;
  t->h_top = top;
  return ok();
}

int finger_descend(const finger_tables* th, const float* queries, int64_t nq, int32_t* out_entries,
                   int32_t* out_calls, void* stream) {
  using namespace finger;
  if (th == nullptr) return fail(FINGER_EINVAL, "NULL handle");
  const Tables* t = reinterpret_cast<const Tables*>(th);
  if (t->h_top < 0) return fail(FINGER_EINVAL, "no upper layers attached (finger_hierarchy_attach)");
  if (nq < 0) return fail(FINGER_EINVAL, "nq < 0");
  if (nq == 0) return ok();
  if (queries == nullptr || out_entries == nullptr) return fail(FINGER_EINVAL, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(queries) & 15u) != 0) return fail(FINGER_EINVAL, "queries must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (t->metric == FINGER_ANGULAR) {
    DevBuf<float> qn;
    int st = dev_alloc(reinterpret_cast<void**>(&qn.p), (size_t)nq * t->m * 4, "normalized queries");
    if (st != FINGER_OK) return st;
    HIPCHK(launch_normalize_rows(queries, nq, t->m, qn.p, s));
    HIPCHK(launch_descend(*t, qn.p, nq, out_entries, out_calls, s));
    HIPCHK(hipStreamSynchronize(s));
    return ok();
  }
  HIPCHK(launch_descend(*t, queries, nq, out_entries, out_calls, s));
  return ok();
}

int finger_estimate_edges(const finger_tables* th, const float* queries, int64_t nq,
                          const int32_t* q_index, const int32_t* centers, const int32_t* slots,
                          int64_t n_items, float* out_est, float* out_t_hat, void* stream) {
  using namespace finger;
  if (th == nullptr) return fail(FINGER_EINVAL, "NULL handle");
  const Tables* t = reinterpret_cast<const Tables*>(th);
  if (t->r == 0) return fail(FINGER_EINVAL, "rank-0 handle has no estimate");
  if (n_items < 0 || nq < 0) return fail(FINGER_EINVAL, "negative size");
  if (n_items == 0) return ok();
  if (!queries || !q_index || !centers || !slots || !out_est || !out_t_hat)
    return fail(FINGER_EINVAL, "NULL pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rpad = rpad_of(t->r);
  DevBuf<float> buf;
  int st = dev_alloc(reinterpret_cast<void**>(&buf.p), (size_t)nq * (rpad + 1) * 4 + 256, "estimate scratch");
  if (st != FINGER_OK) return st;
  Tables tq = *t;
  tq.npiv = 0;  // Pq and |q|^2 only
  float* qq = buf.p;
  float* pq = buf.p + (nq + 63) / 64 * 64;
  DevBuf<float> qn;
  if (t->metric == FINGER_ANGULAR) {
    if ((st = dev_alloc(reinterpret_cast<void**>(&qn.p), (size_t)nq * t->m * 4, "normalized queries")) != FINGER_OK) return st;
    HIPCHK(launch_normalize_rows(queries, nq, t->m, qn.p, s));
    queries = qn.p;
  }
  HIPCHK(launch_query_prep(tq, queries, nq, qq, pq, nullptr, nullptr, s));
  HIPCHK(launch_estimate_edges(*t, queries, qq, pq, q_index, centers, slots, n_items, out_est, out_t_hat, s));
  HIPCHK(hipStreamSynchronize(s));
  return ok();
}

int finger_exact_knn_workspace_size(int64_t n, int32_t m, int64_t nq, int32_t k, size_t* bytes) {
  if (bytes == nullptr) return fail(FINGER_EINVAL, "bytes is NULL");
  if (n <= 0 || m <= 0 || m % 4 != 0 || nq < 0 || k < 1 || k > 128 || k > n)
    return fail(FINGER_EINVAL, "bad sizes (n=%lld m=%d nq=%lld k=%d)", (long long)n, m, (long long)nq, k);
  *bytes = finger::exact_knn_ws_bytes(n, m, nq, k) + align256((size_t)(n + nq) * m * 4);
  return ok();
}

int finger_exact_knn(const float* data, int64_t n, int32_t m, const float* queries, int64_t nq,
                     int32_t k, int32_t metric, int32_t* out_ids, float* out_dist, void* workspace,
                     size_t workspace_bytes, void* stream) {
  using namespace finger;
  size_t need = 0;
  int st = finger_exact_knn_workspace_size(n, m, nq, k, &need);
  if (st != FINGER_OK) return st;
  if (metric != FINGER_L2 && metric != FINGER_ANGULAR && metric != FINGER_IP)
    return fail(FINGER_EINVAL, "unknown metric %d", metric);
  if (nq == 0) return ok();
  if (!data || !queries || !out_ids || !out_dist) return fail(FINGER_EINVAL, "NULL pointer");
  if (((reinterpret_cast<uintptr_t>(data) | reinterpret_cast<uintptr_t>(queries)) & 15u) != 0)
    return fail(FINGER_EINVAL, "data and queries must be 16-byte aligned");
  if (workspace == nullptr || workspace_bytes < need)
    return fail(FINGER_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(FINGER_EINVAL, "workspace must be 256-byte aligned");
  st = check_device(nullptr);
  if (st != FINGER_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const float* X = data;
  const float* Q = queries;
  char* rest = ws + align256((size_t)(n + nq) * m * 4);
  if (metric == FINGER_ANGULAR) {
    float* Xn = reinterpret_cast<float*>(ws);
    float* Qn = Xn + (size_t)n * m;
    HIPCHK(launch_normalize_rows(data, n, m, Xn, s));
    HIPCHK(launch_normalize_rows(queries, nq, m, Qn, s));
    X = Xn;
    Q = Qn;
  }
  HIPCHK(launch_exact_knn(X, n, m, Q, nq, k, metric, out_ids, out_dist, rest, s));
  return ok();
}

// ------------------------------------------------------------------ gate

int64_t finger_gate_param_count(int32_t in_dim, int32_t hidden) {
  if (in_dim < 1 || hidden < 1) return 0;
  return (int64_t)hidden * in_dim + (int64_t)hidden * hidden + 3 * (int64_t)hidden + 1;
}

int finger_gate_attach(finger_tables* th, const float* weights, int32_t in_dim, int32_t hidden,
                       double eps_gate) {
  using namespace finger;
  if (th == nullptr || weights == nullptr) return fail(FINGER_EINVAL, "NULL argument");
  Tables* t = reinterpret_cast<Tables*>(th);
  if (t->r == 0) return fail(FINGER_EINVAL, "rank-0 handle cannot take a gate");
  if (t->metric == FINGER_IP) return fail(FINGER_EINVAL, "the learned gate is for L2 and angular only");
  if (in_dim != FINGER_GATE_FEATURES(t->r))
    return fail(FINGER_EINVAL, "in_dim = %d, expected 2r+4 = %d", in_dim, FINGER_GATE_FEATURES(t->r));
  if (hidden < 1 || hidden > 64) return fail(FINGER_EINVAL, "hidden = %d out of range [1, 64]", hidden);
  const int64_t P = finger_gate_param_count(in_dim, hidden);
  DevBuf<float> wd;
  int st = dev_alloc(reinterpret_cast<void**>(&wd.p), (size_t)P * 4, "gate weights");
  if (st != FINGER_OK) return st;
  HIPCHK(hipMemcpy(wd.p, weights, (size_t)P * 4, hipMemcpyHostToDevice));
  const GateLayout gl = gate_layout(t->r, hidden);
  uint16_t* wbf = nullptr;
  float* b = nullptr;
  if ((st = dev_alloc(reinterpret_cast<void**>(&wbf), (size_t)gl.total * 2, "gate bf16 weights")) != FINGER_OK) return st;
  if ((st = dev_alloc(reinterpret_cast<void**>(&b), (size_t)(2 * gl.hp + 1) * 4, "gate biases")) != FINGER_OK) {
    (void)hipFree(wbf);
    return st;
  }
  hipError_t e = launch_pack_gate(wd.p, in_dim, hidden, wbf, b, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(wbf);
    (void)hipFree(b);
    return fail(FINGER_EDEVICE, "packing gate weights: %s", hipGetErrorString(e));
  }
  if (t->gate_w) (void)hipFree(t->gate_w);
  if (t->gate_b) (void)hipFree(t->gate_b);
  t->gate_w = wbf;
  t->gate_b = b;
  t->gate_in = in_dim;
  t->gate_h = hidden;
  t->eps_gate = eps_gate;
  t->gate = 1;
  return ok();
}

int finger_gate_targets(const float* log_features, const float* log_targets, int64_t rows,
                        int32_t rank, float* out, void* stream) {
  if (!log_features || !log_targets || !out) return fail(FINGER_EINVAL, "NULL pointer");
  if (rows < 0 || rank < 1) return fail(FINGER_EINVAL, "rows < 0 or rank < 1");
  HIPCHK(finger::launch_gate_targets(log_features, log_targets, rows, rank, out,
                                     static_cast<hipStream_t>(stream)));
  return ok();
}

int finger_mlp_forward(const float* weights, int32_t in_dim, int32_t hidden, const float* x,
                       int64_t batch, float* y, void* stream) {
  if (!weights || !x || !y) return fail(FINGER_EINVAL, "NULL pointer");
  if (in_dim < 1 || in_dim > 512 || hidden < 1 || hidden > 64 || batch < 0)
    return fail(FINGER_EINVAL, "bad sizes (1 <= in_dim <= 512, 1 <= hidden <= 64, batch >= 0)");
  HIPCHK(finger::launch_mlp_forward(weights, in_dim, hidden, x, batch, y, static_cast<hipStream_t>(stream)));
  return ok();
}

int finger_mlp_backward_workspace_size(int32_t in_dim, int32_t hidden, int64_t batch, size_t* bytes) {
  if (bytes == nullptr) return fail(FINGER_EINVAL, "NULL pointer");
  if (in_dim < 1 || in_dim > 512 || hidden < 1 || hidden > 64 || batch < 1)
    return fail(FINGER_EINVAL, "bad sizes (1 <= in_dim <= 512, 1 <= hidden <= 64, batch >= 1)");
  *bytes = finger::mlp_backward_scratch_bytes(in_dim, hidden, batch);
  return ok();
}

int finger_mlp_backward(const float* weights, int32_t in_dim, int32_t hidden, const float* x,
                        const float* target, int64_t batch, float* grad, float* loss,
                        void* workspace, size_t workspace_bytes, void* stream) {
  if (!weights || !x || !target || !grad) return fail(FINGER_EINVAL, "NULL pointer");
  if (in_dim < 1 || in_dim > 512 || hidden < 1 || hidden > 64 || batch < 1)
    return fail(FINGER_EINVAL, "bad sizes (1 <= in_dim <= 512, 1 <= hidden <= 64, batch >= 1)");
  const size_t need = finger::mlp_backward_scratch_bytes(in_dim, hidden, batch);
  if (workspace == nullptr || workspace_bytes < need)
    return fail(FINGER_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(FINGER_EINVAL, "workspace must be 256-byte aligned");
  HIPCHK(finger::launch_mlp_backward(weights, in_dim, hidden, x, target, batch, grad, loss, workspace,
                                     static_cast<hipStream_t>(stream)));
  return ok();
}

int finger_gate_calibrate(const float* weights, int32_t in_dim, int32_t hidden, const float* x,
                          const float* target, int64_t rows, double* eps_gate, void* stream) {
  if (!weights || !x || !target || !eps_gate) return fail(FINGER_EINVAL, "NULL pointer");
  if (in_dim < 1 || in_dim > 512 || hidden < 1 || hidden > 64 || rows < 1)
    return fail(FINGER_EINVAL, "bad sizes (1 <= in_dim <= 512, 1 <= hidden <= 64, rows >= 1)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf<float> y;
  int st = dev_alloc(reinterpret_cast<void**>(&y.p), (size_t)rows * 4, "gate outputs");
  if (st != FINGER_OK) return st;
  const int nb = finger::abs_err_blocks(rows);
  DevBuf<double> parts;
  if ((st = dev_alloc(reinterpret_cast<void**>(&parts.p), (size_t)nb * 8, "error sums")) != FINGER_OK) return st;
  HIPCHK(finger::launch_mlp_forward(weights, in_dim, hidden, x, rows, y.p, s));
  HIPCHK(finger::launch_abs_err_parts(y.p, target, rows, parts.p, s));
  std::vector<double> hp((size_t)nb);
  HIPCHK(hipMemcpyAsync(hp.data(), parts.p, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double sum = 0.0;
  for (double v : hp) sum += v;
  *eps_gate = sum / (double)rows;
  return ok();
}

int finger_adam_step(float* weights, const float* grad, float* m1, float* m2, int64_t count,
                     float lr, float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (!weights || !grad || !m1 || !m2) return fail(FINGER_EINVAL, "NULL pointer");
  if (count < 0 || step < 1) return fail(FINGER_EINVAL, "count < 0 or step < 1");
  if (count == 0) return ok();
  HIPCHK(finger::launch_adam(weights, grad, m1, m2, count, lr, beta1, beta2, eps, step,
                             static_cast<hipStream_t>(stream)));
  return ok();
}

}  // extern "C"
