// Checkpoint of a tables handle: finger_tables_export writes every table the
// build produced (basis, distribution-matching constants, node and edge
// tables, pivot operands, build samples, an attached gate) into one
// versioned, checksummed byte image; finger_tables_import rebuilds a handle
// from it over the caller's data and graph, after checking that they are
// the ones the tables were built from.  The paper's own builds take minutes
// (Table 1), which is what this saves.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "../../include/finger.h"
#include "abi_util.h"
#include "internal.h"

using finger::Tables;
using namespace finger::abi;

namespace {

constexpr char kMagic[8] = {'F', 'I', 'N', 'G', 'E', 'R', 'T', 'B'};
constexpr uint32_t kVersion = 1;

// Streaming form of the checksum finger.h documents: four lanes over the
// little-endian 64-bit words of the image (word i feeds lane i mod 4).
struct Checksum {
  uint64_t h[4] = {0x243F6A8885A308D3ull, 0x13198A2E03707344ull, 0xA4093822299F31D0ull,
                   0x082EFA98EC4E6C89ull};
  uint64_t words = 0;
  uint64_t len = 0;
  static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  void word(uint64_t w) {
    uint64_t& x = h[words & 3];
    x = rotl((x ^ w) * 0x9E3779B97F4A7C15ull, 31);
    ++words;
  }
  // bytes must be a multiple of 8 except in the last call
  void update(const void* p, size_t bytes) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
      uint64_t w;
      std::memcpy(&w, b + i, 8);
      word(w);
    }
    if (i < bytes) {
      uint64_t w = 0;
      std::memcpy(&w, b + i, bytes - i);
      word(w);
    }
    len += bytes;
  }
  uint64_t final() const {
    uint64_t x = len;
    for (int j = 0; j < 4; ++j) {
      x = (x ^ h[j]) * 0xBF58476D1CE4E5B9ull;
      x ^= x >> 29;
    }
    return x ^ (x >> 32);
  }
};

// checksum of a device array, streamed through host memory in slices
int device_checksum(const void* dev, size_t bytes, uint64_t* out) {
  Checksum c;
  const size_t slice = (size_t)64 << 20;
  std::vector<unsigned char> buf(std::min(bytes, slice));
  for (size_t off = 0; off < bytes; off += slice) {
    const size_t nb = std::min(slice, bytes - off);
    HIPCHK(hipMemcpy(buf.data(), static_cast<const char*>(dev) + off, nb, hipMemcpyDeviceToHost));
    c.update(buf.data(), nb);
  }
  *out = c.final();
  return FINGER_OK;
}

struct Header {  // the image's first bytes (little-endian, 8-byte fields aligned)
  char magic[8];
  uint32_t version;
  uint32_t n_sections;
  int64_t n;
  int32_t m, r, deg, code_type, metric, sigma_mode, npiv, qprep_cols;
  int32_t gate, gate_in, gate_h, reserved;
  int64_t nsamp;
  double mu, sigma, mu_hat, sigma_hat, eps, corr_xy, eps_gate;
  uint64_t seed;
  uint64_t graph_hash, data_hash;
};

struct Section {
  uint32_t id;
  uint32_t on_host;  // 1: host array of the handle, 0: device array
  uint64_t offset;
  uint64_t bytes;
};

enum SectionId : uint32_t {
  S_P64 = 1, S_EIG, S_P32, S_CC, S_PC, S_ALPHA, S_RHO, S_CODES, S_SCALE, S_SAMPLES, S_XY,
  S_QPREP_B, S_QPREP_BNORM, S_PIV_IDS, S_PIV_B16, S_PIV_NORM, S_GATE_W, S_GATE_B, S_COUNT
};

// Every array of a handle with its size, in a fixed order; `ptr` points at
// the handle's member so that import can allocate into it.
struct Part {
  uint32_t id;
  bool host;
  void** ptr;
  size_t bytes;
};

std::vector<Part> parts_of(Tables* t) {
  using finger::gate_layout;
  using finger::pivot_kpad;
  using finger::pivot_pad_rows;
  const int rpad = finger::rpad_of(t->r);
  const size_t n = (size_t)t->n;
  std::vector<Part> v;
  auto add = [&](uint32_t id, bool host, void* member, size_t bytes) {
    if (bytes > 0) v.push_back({id, host, static_cast<void**>(member), bytes});
  };
  if (t->r > 0) {
    add(S_P64, true, &t->P64_host, (size_t)t->r * t->m * 8);
    add(S_EIG, true, &t->eig_host, (size_t)t->m * 8);
    add(S_P32, false, &t->P, (size_t)rpad * t->m * 4);
  }
  add(S_CC, false, &t->cc, n * 4);
  if (t->r > 0) {
    const size_t esz = t->code_type == FINGER_CODE_F32 ? 4 : (t->code_type == FINGER_CODE_BF16 ? 2 : 1);
    add(S_PC, false, &t->pc, n * rpad * 4);
    add(S_ALPHA, false, &t->alpha, n * t->deg * 4);
    add(S_RHO, false, &t->rho, n * t->deg * 4);
    add(S_CODES, false, &t->codes, n * t->deg * rpad * esz);
    add(S_SCALE, false, &t->scale, n * 4);
    add(S_SAMPLES, false, &t->samples, (size_t)t->nsamp * 12);
    add(S_XY, false, &t->xy, (size_t)t->nsamp * 16);
  }
  if (t->qprep_cols > 0) {
    add(S_QPREP_B, false, &t->qprep_B, (size_t)t->qprep_cols * t->m * 4);
    add(S_QPREP_BNORM, false, &t->qprep_Bnorm, (size_t)t->qprep_cols * 4);
  }
  if (t->npiv > 0) {
    add(S_PIV_IDS, false, &t->piv_ids, (size_t)t->npiv * 4);
    add(S_PIV_B16, false, &t->piv_b16, (size_t)pivot_pad_rows(t->npiv) * pivot_kpad(t->m) * 2);
    add(S_PIV_NORM, false, &t->piv_norm, (size_t)pivot_pad_rows(t->npiv) * 4);
  }
  if (t->gate) {
    const finger::GateLayout gl = gate_layout(t->r, t->gate_h);
    add(S_GATE_W, false, &t->gate_w, (size_t)gl.total * 2);
    add(S_GATE_B, false, &t->gate_b, (size_t)(2 * gl.hp + 1) * 4);
  }
  return v;
}

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" {

uint64_t finger_checksum64(const void* p, size_t bytes) {
  Checksum c;
  if (p != nullptr) c.update(p, bytes);
  return c.final();
}

int finger_tables_export(const finger_tables* th, void* buf, size_t* bytes) {
  if (th == nullptr || bytes == nullptr) return fail(FINGER_EINVAL, "NULL argument");
  Tables* t = const_cast<Tables*>(reinterpret_cast<const Tables*>(th));
  const std::vector<Part> parts = parts_of(t);
  size_t off = round256(sizeof(Header) + parts.size() * sizeof(Section));
  std::vector<Section> secs;
  for (const Part& p : parts) {
    secs.push_back({p.id, p.host ? 1u : 0u, off, p.bytes});
    off = round256(off + p.bytes);
  }
  const size_t total = off + 8;  // trailing checksum
  if (buf == nullptr) {
    *bytes = total;
    return ok();
  }
  if (*bytes < total) {
    const size_t cap = *bytes;
    *bytes = total;
    return fail(FINGER_EOVERFLOW, "the image needs %zu bytes, the buffer has %zu", total, cap);
  }
  *bytes = total;
  HIPCHK(hipSetDevice(t->device));
  char* out = static_cast<char*>(buf);
  std::memset(out, 0, total);
  Header h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.n_sections = (uint32_t)secs.size();
  h.n = t->n;
  h.m = t->m;
  h.r = t->r;
  h.deg = t->deg;
  h.code_type = t->code_type;
  h.metric = t->metric;
  h.sigma_mode = t->sigma_mode;
  h.npiv = t->npiv;
  h.qprep_cols = t->qprep_cols;
  h.gate = t->gate;
  h.gate_in = t->gate_in;
  h.gate_h = t->gate_h;
  h.nsamp = t->nsamp;
  h.mu = t->mu;
  h.sigma = t->sigma;
  h.mu_hat = t->mu_hat;
  h.sigma_hat = t->sigma_hat;
  h.eps = t->eps;
  h.corr_xy = t->corr_xy;
  h.eps_gate = t->eps_gate;
  h.seed = t->seed;
  int st = device_checksum(t->graph, (size_t)t->n * t->deg * 4, &h.graph_hash);
  if (st != FINGER_OK) return st;
  if ((st = device_checksum(t->data, (size_t)t->n * t->m * 4, &h.data_hash)) != FINGER_OK) return st;
  std::memcpy(out, &h, sizeof(h));
  std::memcpy(out + sizeof(h), secs.data(), secs.size() * sizeof(Section));
  for (size_t i = 0; i < parts.size(); ++i) {
    const Part& p = parts[i];
    if (p.host) std::memcpy(out + secs[i].offset, *p.ptr, p.bytes);
    else HIPCHK(hipMemcpy(out + secs[i].offset, *p.ptr, p.bytes, hipMemcpyDeviceToHost));
  }
  const uint64_t sum = finger_checksum64(out, total - 8);
  std::memcpy(out + total - 8, &sum, 8);
  return ok();
}

int finger_tables_import(const void* buf, size_t bytes, const float* data, int64_t n, int32_t m,
                         const int32_t* graph, int32_t max_degree, finger_tables** out,
                         void* stream) {
  using namespace finger;
  if (out == nullptr) return fail(FINGER_EINVAL, "out is NULL");
  *out = nullptr;
  if (buf == nullptr || data == nullptr || graph == nullptr) return fail(FINGER_EINVAL, "NULL argument");
  // ---- host-side checks, before any device call
  const char* in = static_cast<const char*>(buf);
  if (bytes < sizeof(Header) + 8) return fail(FINGER_ECORRUPT, "image of %zu bytes is too short", bytes);
  Header h;
  std::memcpy(&h, in, sizeof(h));
  if (std::memcmp(h.magic, kMagic, 8) != 0) return fail(FINGER_ECORRUPT, "not a FINGER tables image (magic)");
  if (h.version != kVersion) return fail(FINGER_ECORRUPT, "image version %u, this library reads %u", h.version, kVersion);
  uint64_t stored;
  std::memcpy(&stored, in + bytes - 8, 8);
  if (finger_checksum64(in, bytes - 8) != stored) return fail(FINGER_ECORRUPT, "checksum mismatch");
  if (h.n != n || h.m != m || h.deg != max_degree)
    return fail(FINGER_EINVAL, "image is for n = %lld, m = %d, max_degree = %d; got %lld, %d, %d",
                (long long)h.n, h.m, h.deg, (long long)n, m, max_degree);
  if ((reinterpret_cast<uintptr_t>(data) & 15u) != 0) return fail(FINGER_EINVAL, "data must be 16-byte aligned");
  if (h.n_sections > S_COUNT || sizeof(Header) + (size_t)h.n_sections * sizeof(Section) > bytes - 8)
    return fail(FINGER_ECORRUPT, "section table out of range");
  std::vector<Section> secs(h.n_sections);
  std::memcpy(secs.data(), in + sizeof(Header), secs.size() * sizeof(Section));
  if (h.r < 0 || h.r > kMaxRank || h.r > h.m || h.npiv < 0 || h.nsamp < 0 || h.qprep_cols < 0 ||
      h.code_type < FINGER_CODE_F32 || h.code_type > FINGER_CODE_FP8E4M3 ||
      (h.gate && (h.gate_h < 1 || h.gate_h > 64)))
    return fail(FINGER_ECORRUPT, "header fields out of range");
  int dev = 0;
  int st = check_device(&dev);
  if (st != FINGER_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);

  Tables* t = new (std::nothrow) Tables();
  if (t == nullptr) return fail(FINGER_ENOMEM, "host allocation failed");
  Guard guard{t};
  t->device = dev;
  t->n = h.n;
  t->m = h.m;
  t->r = h.r;
  t->deg = h.deg;
  t->code_type = h.code_type;
  t->metric = h.metric;
  t->sigma_mode = h.sigma_mode;
  t->npiv = h.npiv;
  t->qprep_cols = h.qprep_cols;
  t->gate = h.gate;
  t->gate_in = h.gate_in;
  t->gate_h = h.gate_h;
  t->nsamp = h.nsamp;
  t->mu = h.mu;
  t->sigma = h.sigma;
  t->mu_hat = h.mu_hat;
  t->sigma_hat = h.sigma_hat;
  t->eps = h.eps;
  t->corr_xy = h.corr_xy;
  t->eps_gate = h.eps_gate;
  t->seed = h.seed;
  t->graph = graph;
  if (t->metric == FINGER_ANGULAR) {
    if ((st = dev_alloc(reinterpret_cast<void**>(&t->data_owned), (size_t)n * m * 4, "normalized data")) != FINGER_OK) return st;
    HIPCHK(launch_normalize_rows(data, n, m, t->data_owned, s));
    HIPCHK(hipStreamSynchronize(s));
    t->data = t->data_owned;
  } else {
    t->data = data;
  }
  uint64_t gh = 0, dh = 0;
  if ((st = device_checksum(graph, (size_t)n * max_degree * 4, &gh)) != FINGER_OK) return st;
  if (gh != h.graph_hash) return fail(FINGER_EINVAL, "graph differs from the one the tables were built over");
  if ((st = device_checksum(t->data, (size_t)n * m * 4, &dh)) != FINGER_OK) return st;
  if (dh != h.data_hash) return fail(FINGER_EINVAL, "data differ from the points the tables were built over");
  const std::vector<Part> parts = parts_of(t);
  if (parts.size() != secs.size()) return fail(FINGER_ECORRUPT, "image has %zu sections, its header implies %zu", secs.size(), parts.size());
  for (size_t i = 0; i < parts.size(); ++i) {
    const Part& p = parts[i];
    const Section& sc = secs[i];
    if (sc.id != p.id || sc.bytes != p.bytes || (sc.on_host != 0) != p.host || sc.offset > bytes - 8 ||
        sc.bytes > bytes - 8 - sc.offset)
      return fail(FINGER_ECORRUPT, "section %zu (id %u) does not match the header", i, sc.id);
    if (p.host) {
      void* hp = std::malloc(p.bytes);
      if (hp == nullptr) return fail(FINGER_ENOMEM, "host allocation failed");
      std::memcpy(hp, in + sc.offset, p.bytes);
      *p.ptr = hp;
    } else {
      if ((st = dev_alloc(p.ptr, p.bytes, "imported table")) != FINGER_OK) return st;
      HIPCHK(hipMemcpyAsync(*p.ptr, in + sc.offset, p.bytes, hipMemcpyHostToDevice, s));
    }
  }
  if (t->r > 0) {
    const size_t esz = t->code_type == FINGER_CODE_F32 ? 4 : (t->code_type == FINGER_CODE_BF16 ? 2 : 1);
    t->code_bytes = (size_t)t->n * t->deg * finger::rpad_of(t->r) * esz;
  }
  HIPCHK(hipStreamSynchronize(s));
  guard.t = nullptr;
  *out = reinterpret_cast<finger_tables*>(t);
  return ok();
}

}  // extern "C"
