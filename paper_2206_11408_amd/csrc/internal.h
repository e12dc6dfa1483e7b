// Internal declarations of libfinger: the handle layout and the kernel
// launchers each .hip file provides to the C ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/finger.h"

namespace finger {

// Visited set: LDS open-addressing table per query wave, spilling to a
// per-wave global table in the workspace when a probe run gets long.
constexpr int kMaxDegree = 64;
constexpr int kMaxEf = 1024;
constexpr int kMaxRank = 256;
constexpr int kMaxDim = 2048;
constexpr int kDefaultSamples = 100000;

// Per-node and per-edge rows of FINGER's projected tables hold r values
// padded to a multiple of 32 (one 32-element chunk per lane in the search).
inline int rpad_of(int r) { return (r + 31) / 32 * 32; }

// Packed bf16 gate weights (element offsets): W1s [r][hp] | W1e [hp][k1] |
// W2 [hp][k2] | W3 [hp]; hp = hidden rounded up to 16 (MFMA tile), k1 =
// r + 4 rounded up to 32, k2 = hp rounded up to 32.
struct GateLayout {
  int r, hp, k1, k2;
  int64_t w1e, w2, w3, total;
};
__host__ __device__ inline GateLayout gate_layout(int r, int hidden) {
  GateLayout L;
  L.r = r;
  L.hp = (hidden + 15) / 16 * 16;
  L.k1 = (r + 4 + 31) / 32 * 32;
  L.k2 = (L.hp + 31) / 32 * 32;
  L.w1e = (int64_t)r * L.hp;
  L.w2 = L.w1e + (int64_t)L.hp * L.k1;
  L.w3 = L.w2 + (int64_t)L.hp * L.k2;
  L.total = L.w3 + L.hp;
  return L;
}

struct Tables {
  int device = 0;
  int64_t n = 0;
  int32_t m = 0, r = 0, deg = 0, code_type = 0, metric = 0, sigma_mode = 0;
  uint64_t seed = 0;               // build seed of the samples
  const float* data = nullptr;     // points the search reads (borrowed, or data_owned)
  float* data_owned = nullptr;     // normalized copy for FINGER_ANGULAR
  const int32_t* graph = nullptr;  // borrowed
  // basis
  double* P64_host = nullptr;      // [r][m]
  double* eig_host = nullptr;      // [m]
  float* P = nullptr;              // [r][m]
  // node table
  float* cc = nullptr;             // [n]
  float* pc = nullptr;             // [n][r]
  // edge table
  float* alpha = nullptr;          // [n][deg]
  float* rho = nullptr;            // [n][deg]
  void* codes = nullptr;           // [n][deg][r] (f32, bf16 or fp8)
  float* scale = nullptr;          // [n]
  size_t code_bytes = 0;
  // pivots: rows r.. of qprep_B hold the pivot vectors, rows 0..r-1 hold P
  int32_t npiv = 0;
  int32_t* piv_ids = nullptr;      // [npiv]
  float* qprep_B = nullptr;        // [(r + npiv) rounded up to 64][m]
  __bf16* piv_b16 = nullptr;       // [pivot_pad_rows(npiv)][pivot_kpad(m)] pivots in bf16, zero padded
  float* piv_norm = nullptr;       // [pivot_pad_rows(npiv)] |pivot|^2 (fp32), zero padded
  float* qprep_Bnorm = nullptr;    // [(r + npiv) rounded up to 64]  (|row|^2)
  int32_t qprep_cols = 0;          // r + npiv rounded up to 64
  // distribution matching constants
  double mu = 0, sigma = 1, mu_hat = 0, sigma_hat = 1, eps = 0;
  double corr_xy = 0;              // Pearson correlation of the sampled X, Y
  // build samples kept for inspection
  int64_t nsamp = 0;
  int32_t* samples = nullptr;      // [nsamp][3]
  double* xy = nullptr;            // [nsamp][2]
  // learned gate
  int gate = 0;
  int32_t gate_in = 0, gate_h = 0;
  double eps_gate = 0;
  uint16_t* gate_w = nullptr;      // bf16 weights packed as GateLayout
  float* gate_b = nullptr;         // float biases b1 [hp], b2 [hp], b3 [1]
  // upper layers of an HNSW-style hierarchy (finger_hierarchy_attach)
  int32_t h_top = -1;              // descent start: smallest id of the top level
  int32_t h_top_level = 0;
  int32_t h_width = 0;
  int64_t h_rows = 0;
  int32_t* h_row0 = nullptr;       // [n] first upper row of each node (-1: level 0)
  int32_t* h_upper = nullptr;      // [h_rows][h_width]
};

// ------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.

// C[i][j] = sum_k A[i][k] B[j][k] (fp32 MFMA), A [rows][K], B [cols][K];
// epilogue modes below.  rows/cols any size, K % 4 == 0.
enum GemmEpi { GEMM_STORE = 0 };
hipError_t launch_gemm_nt(const float* A, int64_t rows, const float* B, int64_t cols, int K,
                          float* C, int64_t ldc, hipStream_t s);

// greedy descent through the attached upper layers: out[i] = layer-0 start
// point of query i, calls[i] (may be NULL) = distance evaluations
hipError_t launch_descend(const Tables& t, const float* Q, int64_t nq, int32_t* out, int32_t* calls,
                          hipStream_t s);

// flat graph construction (graph.hip); the repair loop runs in api.hip
// kNN lists without the point itself: ids relative to the searched rows,
// self = first + row, written plus id_offset
hipError_t launch_drop_self(const int32_t* ids1, const float* d1, int64_t n, int k1, int k,
                            int32_t* ids, float* dk, int64_t first, int64_t id_offset, hipStream_t s);
hipError_t launch_sym_keys_dst(int64_t n, int k, const int32_t* ids, const float* dk, uint32_t* keys,
                               uint32_t* vals, hipStream_t s);
hipError_t launch_sym_keys_src_d(int64_t n, int k, const int32_t* ids, const float* dk,
                                 const uint32_t* perm, uint64_t* keys, hipStream_t s);
hipError_t launch_sym_dedupe(int64_t n, int k, const int32_t* ids, const float* dk,
                             const uint32_t* perm, uint32_t* flag, uint32_t* cnt, hipStream_t s);
hipError_t launch_sym_fill(int64_t n, int k, const int32_t* ids, const float* dk, const uint32_t* perm,
                           const uint32_t* flag, const uint32_t* pos, int32_t* nbr, float* nd,
                           hipStream_t s);
// hipCUB wrappers: tmp == nullptr queries tmp_bytes
hipError_t radix_sort_u32(void* tmp, size_t& tmp_bytes, const uint32_t* kin, uint32_t* kout,
                          const uint32_t* vin, uint32_t* vout, int64_t count, int end_bit, hipStream_t s);
hipError_t radix_sort_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout,
                          const uint32_t* vin, uint32_t* vout, int64_t count, int end_bit, hipStream_t s);
hipError_t exclusive_sum_u32(void* tmp, size_t& tmp_bytes, const uint32_t* in, uint32_t* out,
                             int64_t count, hipStream_t s);
hipError_t launch_prune(const float* data, int64_t n, int m, const uint32_t* indptr,
                        const int32_t* nbr, const float* nd, int W, int32_t* out, hipStream_t s);
hipError_t launch_degrees(const int32_t* G, int64_t n, int W, int32_t* deg, hipStream_t s);
hipError_t launch_bfs_level(const int32_t* G, int W, const int32_t* frontier, int64_t fsize,
                            uint32_t* reached, int32_t* next, uint32_t* next_count, hipStream_t s);
hipError_t launch_nearest_free(const float* data, int64_t n, int m, int u, const uint32_t* reached,
                               const int32_t* deg, int W, unsigned long long* best, hipStream_t s);

// p[0..count) = value (a kernel, so that callers may capture it in a graph)
hipError_t launch_fill_u32(void* p, uint32_t value, size_t count, hipStream_t s);

// query preparation: qq[i] = |q_i|^2, Pq[i][0..r) = P q_i, and (if npiv > 0)
// entries[i] = nearest pivot id by exact squared distance
hipError_t launch_query_prep(const Tables& t, const float* Q, int64_t nq, float* qq, float* Pq,
                             int32_t* entries, void* scratch, hipStream_t s, bool need_pq = true);
size_t query_prep_scratch_bytes(const Tables& t, int64_t nq);
// bf16 copy of the pivot rows for the query-prep scoring kernel
int pivot_pad_rows(int npiv);
int pivot_kpad(int m);
hipError_t launch_pack_pivots(const float* src, int npiv, int m, __bf16* dst, hipStream_t s);

struct SearchLaunch {
  const float* queries;
  int64_t nq;
  int mode;
  int k_all, ef_all, k_max, ef_max, entry, warmup;
  const int32_t* kq;
  const int32_t* efq;
  const float* qq;
  const float* pq;
  const int32_t* entries;
  int32_t* out_ids;
  float* out_dist;
  int32_t* counters;
  int32_t* queue;
  int32_t* spill;
  int spill_slots_per_wave;
  int vis_cap;
  int vis_probe;    // LDS slots a visited test examines before the spill table
  int waves;        // grid size in waves
  int persistent;
  int prefetch;     // issue every slot's edge code with the adjacency row
  int coalesced;    // FINGER mode: coalesced screen (code rows of 32..256 bytes, degree <= 32)
  float* log_x;
  float* log_y;
  int64_t log_cap;
  int64_t* log_count;
  float gate_band;  // gated mode: band around the bound inside which the gate decides (<= 0: all)
  // one class of an ef-partitioned search: queries qlist[0..*qcount); with
  // nclass > 0 one launch over nclass class lists (stride list_stride),
  // the largest class first
  const int32_t* qlist;
  const int32_t* qcount;
  int nclass;
  int64_t list_stride;
};
hipError_t launch_search(const Tables& t, const SearchLaunch& L, hipStream_t s);

// ef classes of a search with per-query K and ef: class c holds the queries
// whose ef_eff = max(ef, K) is at most bound[c] (and above bound[c - 1]);
// the last class takes everything above
constexpr int kMaxEfClasses = 8;
struct ClassBounds {
  int n;
  int bound[kMaxEfClasses];
};
hipError_t launch_ef_classes(const int32_t* kq, const int32_t* efq, int64_t nq, int k_all, int ef_all,
                             const ClassBounds& cb, int32_t* counts, int32_t* lists, hipStream_t s);
bool search_prefetch_supported(const Tables& t);
int search_lds_bytes(int ef_max, int vis_cap, int r, int m, int gate_in);

hipError_t launch_estimate_edges(const Tables& t, const float* Q, const float* qq,
                                 const float* Pq, const int32_t* qi, const int32_t* ci,
                                 const int32_t* si, int64_t items, float* est, float* that,
                                 hipStream_t s);

// table build
hipError_t launch_validate_graph(const int32_t* graph, int64_t n, int deg, int32_t* bad,
                                 hipStream_t s);
hipError_t launch_sample_pairs(const int32_t* graph, int64_t n, int deg, int64_t ns,
                               uint64_t seed, int32_t* samples, hipStream_t s);
hipError_t launch_residuals_f64(const float* data, int m, const int32_t* samples, int64_t ns,
                                double* res1, double* res2, hipStream_t s);
int gram_parts(int64_t ns, int m);
hipError_t launch_gram_f64(const double* R, int64_t ns, int m, double* M, hipStream_t s);
hipError_t launch_pair_cosines(const double* res1, const double* res2, int64_t ns, int m,
                               const double* P64, int r, double* xy, hipStream_t s);
hipError_t launch_dm_sums(const double* xy, int64_t ns, double mu, double mu_hat,
                          double scale, int stage, double* out, hipStream_t s);
hipError_t launch_row_norms(const float* X, int64_t n, int m, float* out, hipStream_t s);
hipError_t launch_edge_codes(const Tables& t, hipStream_t s);
hipError_t launch_normalize_rows(const float* X, int64_t n, int m, float* Y, hipStream_t s);
hipError_t launch_gather_rows(const float* X, int m, const int32_t* ids, int64_t cnt, float* Y,
                              hipStream_t s);
hipError_t launch_check_ids(const int32_t* ids, int64_t cnt, int64_t n, int32_t* bad,
                            hipStream_t s);

// exact kNN
size_t exact_knn_ws_bytes(int64_t n, int m, int64_t nq, int k);
hipError_t launch_exact_knn(const float* data, int64_t n, int m, const float* Q, int64_t nq,
                            int k, int metric, int32_t* ids, float* dist, void* ws,
                            hipStream_t s);

// gate
hipError_t launch_mlp_forward(const float* w, int in, int H, const float* x, int64_t B, float* y,
                              hipStream_t s);
size_t mlp_backward_scratch_bytes(int in, int H, int64_t B);
hipError_t launch_mlp_backward(const float* w, int in, int H, const float* x, const float* tgt,
                               int64_t B, float* grad, float* loss, void* scratch, hipStream_t s);
// per-block float64 sums of |t - y| (abs_err_blocks(rows) of them)
int abs_err_blocks(int64_t rows);
hipError_t launch_abs_err_parts(const float* y, const float* t, int64_t rows, double* parts,
                                hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m1, float* m2, int64_t cnt, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s);
hipError_t launch_gate_targets(const float* x, const float* y, int64_t rows, int r, float* out,
                               hipStream_t s);
hipError_t launch_pack_gate(const float* w_dev, int in, int H, uint16_t* wbf, float* b,
                            hipStream_t s);

// host symmetric eigensolver (cyclic Jacobi), eigenvalues descending,
// eigenvectors as rows of V [m][m]
void eigh_jacobi(const double* A, int m, double* evals, double* V);

}  // namespace finger
