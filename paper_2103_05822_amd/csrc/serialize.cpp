// Handle serialisation: the FP64 factors, ranks and box grid of a Tucker handle in a
// binary file, so a long setup (far-field fill + HOSVD) is done once.
//
// File layout, little-endian, every field 8-byte aligned:
//   char[8]  magic "TUCKFMM\1"
//   int64    version (1)
//   int64    n_theta, n_phi, n_groups
//   int64    offsets[n_groups + 1]
//   int64    n_boxes (0: group-compact layout), kx, ky, kz, box[n_groups] if n_boxes > 0
//   per (group, alpha) in order 2 g + alpha:
//     int64  r_theta, r_phi, r_beta, ident
//     complex128 core[r_theta r_phi r_beta], U^theta[n_theta r_theta], U^phi[n_phi r_phi],
//                U^beta[n_beta r_beta]     (the shapes of fmm_tucker_set_group)
//   int64    checksum: the sum of all preceding 8-byte words, modulo 2^64
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>

#include "internal.hpp"

using namespace tuckfmm;

namespace {

constexpr char kMagic[8] = {'T', 'U', 'C', 'K', 'F', 'M', 'M', 1};
constexpr int64_t kVersion = 1;

struct FileCloser {
  void operator()(FILE* f) const {
    if (f) std::fclose(f);
  }
};
using File = std::unique_ptr<FILE, FileCloser>;

// Writes 8-byte words and keeps the running checksum.
struct Writer {
  FILE* f;
  uint64_t sum = 0;
  bool ok = true;
  void words(const void* p, size_t n) {
    if (!ok || n == 0) return;
    const uint64_t* w = static_cast<const uint64_t*>(p);
    for (size_t i = 0; i < n; ++i) sum += w[i];
    ok = std::fwrite(p, 8, n, f) == n;
  }
  void i64(int64_t v) { words(&v, 1); }
};

struct Reader {
  FILE* f;
  uint64_t sum = 0;
  bool ok = true;
  void words(void* p, size_t n) {
    if (!ok || n == 0) return;
    ok = std::fread(p, 8, n, f) == n;
    if (!ok) return;
    const uint64_t* w = static_cast<const uint64_t*>(p);
    for (size_t i = 0; i < n; ++i) sum += w[i];
  }
  int64_t i64() {
    int64_t v = 0;
    words(&v, 1);
    return ok ? v : -1;
  }
};

}  // namespace

extern "C" fmm_status fmm_tucker_save(fmm_tucker_t h, const char* path) {
  clear_error();
  if (!h || !path) return fail(FMM_ERR_ARG, "handle and path must be non-NULL");
  const Layout& L = h->layout;
  for (int i = 0; i < 2 * L.n_groups; ++i)
    if (!h->t[i].set()) return fail(FMM_ERR_STATE, "factors of group %d polarisation %d are not set", i / 2, i % 2);
  File f(std::fopen(path, "wb"));
  if (!f) return fail(FMM_ERR_IO, "cannot open %s for writing", path);
  Writer w{f.get()};
  w.words(kMagic, 1);
  w.i64(kVersion);
  w.i64(L.n_theta);
  w.i64(L.n_phi);
  w.i64(L.n_groups);
  w.words(L.offsets.data(), L.offsets.size());
  w.i64(h->n_boxes);
  if (h->n_boxes > 0) {
    for (int c = 0; c < 3; ++c) w.i64(h->box_dims[c]);
    w.words(h->box.data(), h->box.size());
  } else {
    for (int c = 0; c < 3; ++c) w.i64(0);
  }
  static_assert(sizeof(cd) == 16, "complex128");
  for (const TensorFactors& tf : h->t) {
    w.i64(tf.rt);
    w.i64(tf.rp);
    w.i64(tf.rb);
    w.i64(tf.ident ? 1 : 0);
    for (const std::vector<cd>* v : {&tf.core, &tf.ut, &tf.up, &tf.ub}) w.words(v->data(), 2 * v->size());
  }
  const uint64_t sum = w.sum;
  w.words(&sum, 1);
  if (!w.ok || std::fflush(f.get()) != 0) return fail(FMM_ERR_IO, "write to %s failed", path);
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_load(const char* path, fmm_tucker_t* out) {
  clear_error();
  if (!path || !out) return fail(FMM_ERR_ARG, "path and out must be non-NULL");
  *out = nullptr;
  File f(std::fopen(path, "rb"));
  if (!f) return fail(FMM_ERR_IO, "cannot open %s", path);
  Reader r{f.get()};
  char magic[8];
  r.words(magic, 1);
  if (!r.ok || std::memcmp(magic, kMagic, 8) != 0) return fail(FMM_ERR_IO, "%s is not a tuckfmm handle file", path);
  if (r.i64() != kVersion) return fail(FMM_ERR_IO, "%s: unsupported version", path);
  const int64_t nt = r.i64(), np = r.i64(), ng = r.i64();
  if (!r.ok || nt < 1 || np < 1 || ng < 1 || nt > 1 << 16 || np > 1 << 16 || ng > INT32_MAX / 2)
    return fail(FMM_ERR_IO, "%s: bad header", path);
  std::vector<int64_t> offsets((size_t)ng + 1);
  r.words(offsets.data(), offsets.size());
  if (!r.ok) return fail(FMM_ERR_IO, "%s: truncated", path);
  fmm_layout lay{(int32_t)nt, (int32_t)np, (int32_t)ng, 0, offsets.data()};
  fmm_tucker_t h = nullptr;
  fmm_status st = fmm_tucker_create(&lay, &h);
  if (st != FMM_OK) {
    const std::string why = fmm_last_error();
    return fail(FMM_ERR_IO, "%s: bad layout (%s)", path, why.c_str());
  }
  std::unique_ptr<fmm_tucker_s, void (*)(fmm_tucker_t)> guard(h, fmm_tucker_destroy);
  const int64_t nbox = r.i64();
  int64_t dims[3];
  for (int c = 0; c < 3; ++c) dims[c] = r.i64();
  std::vector<int64_t> box;
  if (r.ok && nbox > 0) {
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || dims[0] * dims[1] * dims[2] != nbox || nbox > (int64_t)1 << 30)
      return fail(FMM_ERR_IO, "%s: bad box grid", path);
    box.resize((size_t)ng);
    r.words(box.data(), box.size());
  }
  if (!r.ok) return fail(FMM_ERR_IO, "%s: truncated", path);
  const Layout& L = h->layout;
  for (int64_t i = 0; i < 2 * ng; ++i) {
    const int g = (int)(i / 2);
    const int64_t rt = r.i64(), rp = r.i64(), rb = r.i64(), ident = r.i64();
    if (!r.ok) return fail(FMM_ERR_IO, "%s: truncated", path);
    if (rt < 1 || rt > nt || rp < 1 || rp > np || rb < 1 || rb > L.nb(g) || (ident != 0 && ident != 1))
      return fail(FMM_ERR_IO, "%s: bad ranks of group %d", path, g);
    TensorFactors tf;
    tf.rt = (int32_t)rt;
    tf.rp = (int32_t)rp;
    tf.rb = (int32_t)rb;
    tf.ident = ident == 1;
    tf.core.resize((size_t)(rt * rp * rb));
    tf.ut.resize((size_t)(nt * rt));
    tf.up.resize((size_t)(np * rp));
    tf.ub.resize((size_t)L.nb(g) * rb);
    for (std::vector<cd>* v : {&tf.core, &tf.ut, &tf.up, &tf.ub}) r.words(v->data(), 2 * v->size());
    if (!r.ok) return fail(FMM_ERR_IO, "%s: truncated", path);
    if (tf.ident) {  // the flag must describe the factors: exact identities
      bool eye = rt == nt && rp == np;
      for (int64_t a = 0; eye && a < nt * nt; ++a) eye = tf.ut[(size_t)a] == cd(a % (nt + 1) == 0 ? 1.0 : 0.0, 0.0);
      for (int64_t a = 0; eye && a < np * np; ++a) eye = tf.up[(size_t)a] == cd(a % (np + 1) == 0 ? 1.0 : 0.0, 0.0);
      if (!eye) return fail(FMM_ERR_IO, "%s: group %d marked identity with other factors", path, g);
    }
    h->t[(size_t)i] = std::move(tf);
  }
  const uint64_t want = r.sum;
  uint64_t got = 0;
  r.words(&got, 1);
  if (!r.ok || got != want) return fail(FMM_ERR_IO, "%s: checksum mismatch", path);
  if (nbox > 0) {
    st = fmm_tucker_set_box_grid(h, (int32_t)dims[0], (int32_t)dims[1], (int32_t)dims[2], box.data());
    if (st != FMM_OK) {
      const std::string why = fmm_last_error();
      return fail(FMM_ERR_IO, "%s: bad box grid (%s)", path, why.c_str());
    }
  }
  *out = guard.release();
  return FMM_OK;
}
