// C ABI entry points: argument validation, handles, arena packing and kernel
// dispatch for the Tucker and dense paths.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.hpp"
#include "kernels.hpp"

// hash of the kernel sources, set by the build
#ifndef TUCKFMM_SOURCE_SHA
#define TUCKFMM_SOURCE_SHA "unknown"
#endif

namespace tuckfmm {

namespace {
thread_local std::string g_err;
}

fmm_status fail(fmm_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void clear_error() { g_err.clear(); }

const char* last_error_cstr() { return g_err.c_str(); }

bool have_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    fail(FMM_ERR_DEVICE, "no HIP device available");
    return false;
  }
  return true;
}

fmm_status copy_layout(const fmm_layout* in, Layout* out) {
  if (!in) return fail(FMM_ERR_ARG, "layout is NULL");
  if (in->reserved != 0) return fail(FMM_ERR_ARG, "layout.reserved must be 0");
  if (in->n_theta < 1 || in->n_phi < 1 || (int64_t)in->n_theta * in->n_phi > (1 << 24))
    return fail(FMM_ERR_SHAPE, "n_theta=%d n_phi=%d out of range", in->n_theta, in->n_phi);
  if (in->n_groups < 0) return fail(FMM_ERR_SHAPE, "n_groups must be >= 0");
  if (!in->offsets) return fail(FMM_ERR_ARG, "layout.offsets is NULL");
  if (in->offsets[0] != 0) return fail(FMM_ERR_SHAPE, "offsets[0] must be 0");
  for (int32_t g = 0; g < in->n_groups; ++g) {
    const int64_t nb = in->offsets[g + 1] - in->offsets[g];
    if (nb < 1) return fail(FMM_ERR_SHAPE, "group %d is empty or offsets decrease", g);
    if (nb > (1 << 24)) return fail(FMM_ERR_SHAPE, "group %d has too many basis functions", g);
  }
  out->n_theta = in->n_theta;
  out->n_phi = in->n_phi;
  out->n_groups = in->n_groups;
  out->offsets.assign(in->offsets, in->offsets + in->n_groups + 1);
  return FMM_OK;
}

}  // namespace tuckfmm

using namespace tuckfmm;

namespace {

// Every precision but FMM_C128 stores complex64 factors and takes complex64 vectors.
size_t elem_bytes(fmm_prec p) { return p == FMM_C128 ? 16 : 8; }
int pack_elems(fmm_prec p) { return p == FMM_C128 ? 1 : 2; }
bool prec_valid(int p) { return p >= FMM_C128 && p <= FMM_BF16X3; }
bool prec_is_split(fmm_prec p) { return p == FMM_BF16X2 || p == FMM_BF16X3; }

// Smallest even nrhs for which FMM_C64 and FMM_C128 take the matrix-core products
// when untuned.  With two right-hand sides the matrix-core pass already beats the
// streaming kernels, which read the factors once per right-hand side (30-lambda
// sphere: FP32 2.70 against 3.83 ms, FP64 5.22 against 7.42 ms).
constexpr int kMfmaMinRhs = 2;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool aligned(const void* p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; }

// Device layout of one precision slot, computed identically for sizing and packing:
// [header: items, work list, pass list][factors].
struct ArenaPlan {
  size_t header_bytes = 0, factor_bytes = 0, total_bytes = 0, factor_bytes_paper = 0;
  std::vector<TuckItem> items;
  std::vector<TuckUnit> units;
  std::vector<TuckSplit> splits;
  int64_t part_stride = 0;
  std::vector<int32_t> order, pass, zero_rows;
  TuckMax mx{};
};

// Bytes streamed by one item (U^beta and the core), the key of the work lists.
double item_cost(const TuckItem& it) { return (double)it.rb * ((double)it.ld_ub + (double)it.ld_c); }

// A layout of few large groups leaves most of the GPU idle with one workgroup per
// item (the trihedral at 2 lambda has 38 items).  Below kSplitBelow items, items
// streaming more than max(kSplitMin, total / kSplitUnits) elements run as blocks of
// their r_beta rows on several workgroups.  With more items splitting only adds
// partial-sum traffic and a finishing launch: measured on MI355X, 196 items of the
// 20-lambda sphere at 4-lambda boxes ran 1.49 ms unsplit and 1.91 ms split.
constexpr int kSplitBelow = 128;
constexpr double kSplitMin = 65536.0;
constexpr double kSplitUnits = 512.0;
constexpr int kSplitMinRows = 4;

// LDS of one CU (gfx950), and the fewest wavefronts per CU with which the streaming
// kernels stage the angular operands in LDS.
constexpr size_t kCuLds = 160 * 1024;
constexpr int kStageMinWaves = 8;

double split_elems(const std::vector<TuckItem>& items) {
  if (const char* env = std::getenv("TUCKFMM_SPLIT_ELEMS")) {
    const double v = std::atof(env);
    if (v >= 1.0) return v;
  }
  if ((int)items.size() >= kSplitBelow) return 1e300;
  double total = 0.0;
  for (const TuckItem& it : items) total += item_cost(it);
  return std::max(kSplitMin, total / kSplitUnits);
}

fmm_status plan_arena(const fmm_tucker_s* h, fmm_prec prec, ArenaPlan* P) {
  const Layout& L = h->layout;
  const int G = L.n_groups;
  const size_t es = elem_bytes(prec);
  const int E = pack_elems(prec);
  const size_t blk_align = 256;
  P->items.resize((size_t)2 * G);
  size_t off = 0;  // bytes inside the factor area
  auto block = [&](size_t n_el) {
    const size_t start = off;
    off = align_up(off + n_el * es, blk_align);
    return start;
  };
  TuckMax mx{};
  for (int g = 0; g < G; ++g) {
    for (int a = 0; a < 2; ++a) {
      const TensorFactors& tf = h->t[2 * g + a];
      if (!tf.set()) return fail(FMM_ERR_STATE, "factors of group %d polarisation %d are not set", g, a);
      TuckItem it{};
      it.nb = L.nb(g);
      it.rt = tf.rt;
      it.rp = tf.rp;
      it.rb = tf.rb;
      it.ld_ub = (it.nb + E - 1) / E * E;
      it.ld_c = (it.rt * it.rp + E - 1) / E * E;
      it.group = g;
      it.alpha = a;
      it.frow = h->box.empty() ? 2 * g + a : (int32_t)(a * h->n_boxes + h->box[g]);
      it.row0 = L.offsets[g];
      // both orders of the two angular products; take the cheaper one
      const double c_theta = (double)L.n_theta * it.rp * (it.rt + L.n_phi);
      const double c_phi = (double)it.rt * L.n_phi * (it.rp + L.n_theta);
      it.theta_first = c_theta <= c_phi ? 1 : 0;
      it.ident = tf.ident ? 1 : 0;
      it.off_ubt = (int64_t)(block((size_t)it.rb * it.ld_ub) / es);
      it.off_core = (int64_t)(block((size_t)it.rb * it.ld_c) / es);
      if (!it.ident) {  // identity angular factors are not stored
        it.off_ut = (int64_t)(block((size_t)L.n_theta * it.rt) / es);
        it.off_up = (int64_t)(block((size_t)L.n_phi * it.rp) / es);
        it.off_upt = (int64_t)(block((size_t)L.n_phi * it.rp) / es);
      }
      P->items[2 * g + a] = it;
      mx.nb = std::max(mx.nb, it.nb);
      mx.rt = std::max(mx.rt, it.rt);
      mx.rp = std::max(mx.rp, it.rp);
      mx.rb = std::max(mx.rb, it.rb);
      mx.q = std::max(mx.q, it.rt * it.rp);
      if (!it.ident) mx.t3 = std::max(mx.t3, it.theta_first ? L.n_theta * it.rp : it.rt * L.n_phi);
      P->factor_bytes_paper +=
          it.ident ? es * ((size_t)it.rt * it.rp * it.rb + (size_t)it.nb * it.rb)   // W and U^beta
                   : es * ((size_t)it.rt * it.rp * it.rb + (size_t)L.n_theta * it.rt + (size_t)L.n_phi * it.rp +
                           (size_t)it.nb * it.rb);
    }
  }
  mx.nt = L.n_theta;
  mx.np = L.n_phi;
  mx.stage = 0;  // decided at upload, with the workgroup size
  P->mx = mx;
  // work units: whole items, or row blocks of the items above the split size
  const double split = split_elems(P->items);
  int64_t agg_off = 0, dis_off = 0;
  std::vector<double> ucost;
  for (int i = 0; i < 2 * G; ++i) {
    const TuckItem& it = P->items[i];
    const double c = item_cost(it);
    int parts = (int)std::min<double>(std::ceil(c / split), (it.rb + kSplitMinRows - 1) / kSplitMinRows);
    if (parts > 1) {
      const int rows = (it.rb + parts - 1) / parts;
      parts = (it.rb + rows - 1) / rows;
      TuckSplit sp{};
      sp.item = i;
      sp.n_parts = parts;
      sp.q_pad = (it.rt * it.rp + 1) / 2 * 2;
      sp.nb_pad = (it.nb + 1) / 2 * 2;
      sp.agg_off = agg_off;
      sp.dis_off = dis_off;
      agg_off += (int64_t)parts * sp.q_pad;
      dis_off += (int64_t)parts * sp.nb_pad;
      const int j = (int)P->splits.size();
      P->splits.push_back(sp);
      for (int s = 0; s < parts; ++s) {
        const int b0 = s * rows, b1 = std::min(it.rb, b0 + rows);
        P->units.push_back(TuckUnit{i, b0, b1, j, s, 0});
        ucost.push_back(c * (b1 - b0) / it.rb);
      }
    } else {
      P->units.push_back(TuckUnit{i, 0, it.rb, -1, 0, 0});
      ucost.push_back(c);
    }
  }
  for (TuckSplit& sp : P->splits) sp.dis_off += agg_off;  // one buffer: agg blocks, then dis blocks
  P->part_stride = (agg_off + dis_off + 31) / 32 * 32;
  // work lists in longest-processing-time order
  const int n = (int)P->units.size();
  P->order.resize(n);
  std::iota(P->order.begin(), P->order.end(), 0);
  std::stable_sort(P->order.begin(), P->order.end(), [&](int32_t a, int32_t b) { return ucost[a] > ucost[b]; });
  // The pass list takes the aggregation and the disaggregation of the i-th largest
  // unit in turn.  Workgroups go to the eight XCDs round-robin by index, so with the
  // pair always in the same order the even XCDs would run only aggregation units and
  // the odd ones only disaggregation units, which take longer on small boxes (the 0.5-
  // lambda layout of the 20-lambda sphere: the two halves of the chip finished 623 and
  // 900 us into the pass).  Every other group of four pairs is therefore swapped.
  P->pass.resize((size_t)2 * n);
  for (int i = 0; i < n; ++i) {
    const int first = (i / 4) & 1;
    P->pass[2 * i + first] = P->order[i];        // aggregation of the i-th largest unit
    P->pass[2 * i + 1 - first] = ~P->order[i];   // and its disaggregation
  }
  // box grid: the rows of the empty boxes, written zero by the aggregation
  if (!h->box.empty()) {
    std::vector<char> used((size_t)h->n_boxes, 0);
    for (int64_t b : h->box) used[(size_t)b] = 1;
    for (int a = 0; a < 2; ++a)
      for (int64_t b = 0; b < h->n_boxes; ++b)
        if (!used[(size_t)b]) P->zero_rows.push_back((int32_t)(a * h->n_boxes + b));
  }
  P->header_bytes = align_up(P->items.size() * sizeof(TuckItem) + P->units.size() * sizeof(TuckUnit) +
                                 P->splits.size() * sizeof(TuckSplit) +
                                 (P->order.size() + P->pass.size() + P->zero_rows.size()) * sizeof(int32_t),
                             256);
  P->factor_bytes = off;
  P->total_bytes = P->header_bytes + P->factor_bytes;
  return FMM_OK;
}

template <typename S>
void put(S* dst, const cd& v);
template <>
void put<double>(double* dst, const cd& v) {
  dst[0] = v.real();
  dst[1] = v.imag();
}
template <>
void put<float>(float* dst, const cd& v) {
  dst[0] = (float)v.real();
  dst[1] = (float)v.imag();
}

template <typename S>
void pack_tensor(const Layout& L, const TensorFactors& tf, const TuckItem& it, S* fac) {
  const int nt = L.n_theta, np = L.n_phi;
  S* ubt = fac + 2 * it.off_ubt;
  for (int n = 0; n < it.nb; ++n)
    for (int b = 0; b < it.rb; ++b) put<S>(ubt + 2 * ((size_t)b * it.ld_ub + n), tf.ub[(size_t)n * it.rb + b]);
  S* core = fac + 2 * it.off_core;
  for (int a = 0; a < it.rt; ++a)
    for (int c = 0; c < it.rp; ++c)
      for (int b = 0; b < it.rb; ++b)
        put<S>(core + 2 * ((size_t)b * it.ld_c + a * it.rp + c), tf.core[((size_t)a * it.rp + c) * it.rb + b]);
  if (it.ident) return;
  S* ut = fac + 2 * it.off_ut;
  for (size_t i = 0; i < (size_t)nt * it.rt; ++i) put<S>(ut + 2 * i, tf.ut[i]);
  S* up = fac + 2 * it.off_up;
  for (size_t i = 0; i < (size_t)np * it.rp; ++i) put<S>(up + 2 * i, tf.up[i]);
  S* upt = fac + 2 * it.off_upt;
  for (int j = 0; j < np; ++j)
    for (int c = 0; c < it.rp; ++c) put<S>(upt + 2 * ((size_t)c * np + j), tf.up[(size_t)j * it.rp + c]);
}

fmm_status check_vec(const void* p, size_t align, const char* name) {
  if (!p) return fail(FMM_ERR_ARG, "%s is NULL", name);
  if (!aligned(p, align)) return fail(FMM_ERR_ARG, "%s must be %zu-byte aligned", name, align);
  return FMM_OK;
}

fmm_status ready_slot(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, PrecSlot** out) {
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  if (!prec_valid(prec)) return fail(FMM_ERR_ARG, "bad precision %d", (int)prec);
  if (nrhs < 1 || nrhs > 65535) return fail(FMM_ERR_ARG, "nrhs must be in [1, 65535]");
  PrecSlot& s = h->slot[prec];
  if (!s.ready) return fail(FMM_ERR_STATE, "precision %d has not been uploaded", (int)prec);
  if (!have_device()) return FMM_ERR_DEVICE;
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));
  if (dev != s.device) return fail(FMM_ERR_STATE, "current device %d differs from the arena's device %d", dev, s.device);
  *out = &s;
  return FMM_OK;
}

fmm_status lds_check(size_t bytes) {
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));
  int lim = 0;
  TFMM_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (bytes > (size_t)lim)
    return fail(FMM_ERR_UNSUPPORTED, "kernel needs %zu bytes of LDS, device allows %d", bytes, lim);
  return FMM_OK;
}

// Which kernels run a call with nrhs right-hand sides.
struct Route {
  bool mfma = false;  // matrix-core products (else the streaming kernels)
  int variant = 0;    // grouped GEMM arithmetic: 0 FP32, 1 BF16x2, 2 BF16x3, 3 FP64
  int tile_steps = 0, rhs_chunk = 0, order = 0;
  int threads = 512;  // streaming kernels' workgroup size
};

// Whether the matrix-core path may run nrhs right-hand sides.  Its paired 16-byte
// loads read factor rows only, and vector operands are loaded and stored one value at
// a time, so FMM_C64 and FMM_C128 take any nrhs (an odd one when tuned so, or for
// FMM_C128 when its items do not fit the streaming kernels); the bf16 split
// precisions are defined for an even nrhs.
bool mfma_allows(fmm_prec prec, int nrhs) { return !prec_is_split(prec) || nrhs % 2 == 0; }

fmm_status route_of(const PrecSlot& s, fmm_prec prec, int nrhs, Route* r) {
  *r = Route{};
  r->threads = s.threads;
  for (const TuneChoice& t : s.tuned)
    if (t.nrhs == nrhs && t.path == 0 && t.threads) r->threads = t.threads;
  if (prec_is_split(prec)) {
    if (nrhs % 2) return fail(FMM_ERR_UNSUPPORTED, "the bf16 split precisions need an even nrhs");
    r->mfma = true;
    r->variant = prec == FMM_BF16X2 ? 1 : 2;
  } else {
    r->mfma = nrhs % 2 == 0 && nrhs >= kMfmaMinRhs;
    r->variant = prec == FMM_C128 ? 3 : 0;
  }
  for (const TuneChoice& t : s.tuned)
    if (t.nrhs == nrhs) {
      r->mfma = t.path == 1;
      r->tile_steps = t.tile_steps;
      r->rhs_chunk = t.rhs_chunk;
      r->order = t.order;
    }
  // FP64 items too large for the streaming kernels' LDS (an item's x_g or core-stage
  // vector plus its r_beta or angular intermediate, in complex128) run on the matrix
  // cores at any nrhs
  if (prec == FMM_C128 && !r->mfma && !s.streams) r->mfma = true;
  return FMM_OK;
}

// Drops a captured graph (it may point at tables or factors about to change).
void drop_graph(fmm_tucker_t h);

// Work counter of the pass kernel (allocated once) and partial-sum buffer of the split
// items for nrhs right-hand sides (grown on demand; a graph captured with the old
// buffer is dropped).
fmm_status ensure_part(fmm_tucker_t h, PrecSlot& s, fmm_prec prec, int nrhs) {
  if (!s.next) TFMM_HIP(hipMalloc(&s.next, 256));
  s.plan.next = s.next;
  if (s.plan.n_splits == 0) return FMM_OK;
  const size_t need = (size_t)s.plan.part_stride * nrhs * elem_bytes(prec);
  if (need > s.part_bytes) {
    drop_graph(h);
    if (s.part) (void)hipFree(s.part);
    s.part = nullptr;
    s.part_bytes = 0;
    TFMM_HIP(hipMalloc(&s.part, need));
    s.part_bytes = need;
  }
  s.plan.part = s.part;
  return FMM_OK;
}

void part_release(PrecSlot& s) {
  if (s.part) (void)hipFree(s.part);
  if (s.next) (void)hipFree(s.next);
  s.part = nullptr;
  s.part_bytes = 0;
  s.next = nullptr;
  s.plan.part = nullptr;
  s.plan.next = nullptr;
}

// Launches one stage (0 aggregation, 1 disaggregation, 2 both) for a validated call.
fmm_status run_stage(fmm_tucker_t h, PrecSlot& s, fmm_prec prec, int nrhs, int stage, const void* x, void* F,
                     const void* G, void* V, hipStream_t hs) {
  const Layout& L = h->layout;
  Route r;
  fmm_status st = route_of(s, prec, nrhs, &r);
  if (st != FMM_OK) return st;
  if (stage != 1 && s.plan.n_zero_rows > 0)  // box grid: F is zero on empty boxes (eq. (3))
    TFMM_HIP(launch_zero_rows(elem_bytes(prec), F, s.plan.zero_rows, s.plan.n_zero_rows,
                              (int64_t)L.ndir() * nrhs, hs));
  if (r.mfma) {
    // vector values are loaded and stored one complex value at a time (the paired
    // 16-byte loads read factor rows only): natural alignment, checked by the callers,
    // is all the matrix-core path needs
    MrhsPlan* mp = nullptr;
    if ((st = mrhs_get(s, elem_bytes(prec), L, nrhs, r.tile_steps, r.rhs_chunk, r.order, &mp)) != FMM_OK) return st;
    return mrhs_run(*mp, s, r.variant, elem_bytes(prec), stage, x, F, G, V, hs);
  }
  if ((st = ensure_part(h, s, prec, nrhs)) != FMM_OK) return st;
  if (prec == FMM_C128) {
    if ((st = lds_check(tucker_lds_bytes<double>(s.plan.mx))) != FMM_OK) return st;
    if (stage == 0) TFMM_HIP(launch_tucker_agg<double>(s.plan, r.threads, L.n_theta, L.n_phi, nrhs, x, F, hs));
    if (stage == 1) TFMM_HIP(launch_tucker_disagg<double>(s.plan, r.threads, L.n_theta, L.n_phi, nrhs, G, V, hs));
    if (stage == 2) TFMM_HIP(launch_tucker_pass<double>(s.plan, r.threads, L.n_theta, L.n_phi, nrhs, x, F, G, V, hs));
  } else {
    if ((st = lds_check(tucker_lds_bytes<float>(s.plan.mx))) != FMM_OK) return st;
    if (stage == 0) TFMM_HIP(launch_tucker_agg<float>(s.plan, r.threads, L.n_theta, L.n_phi, nrhs, x, F, hs));
    if (stage == 1) TFMM_HIP(launch_tucker_disagg<float>(s.plan, r.threads, L.n_theta, L.n_phi, nrhs, G, V, hs));
    if (stage == 2) TFMM_HIP(launch_tucker_pass<float>(s.plan, r.threads, L.n_theta, L.n_phi, nrhs, x, F, G, V, hs));
  }
  return FMM_OK;
}

void drop_graph(fmm_tucker_t h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
}

}  // namespace

// ----------------------------------------------------------------------- misc

extern "C" const char* fmm_last_error(void) { return tuckfmm::last_error_cstr(); }

extern "C" const char* fmm_version(void) { return "tuckfmm 0.2 gfx950 src " TUCKFMM_SOURCE_SHA; }

extern "C" int32_t fmm_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

// --------------------------------------------------------------------- Tucker

extern "C" fmm_status fmm_tucker_create(const fmm_layout* layout, fmm_tucker_t* out) {
  clear_error();
  if (!out) return fail(FMM_ERR_ARG, "out is NULL");
  *out = nullptr;
  auto* h = new fmm_tucker_s();
  fmm_status st = copy_layout(layout, &h->layout);
  if (st != FMM_OK) {
    delete h;
    return st;
  }
  h->t.resize((size_t)2 * h->layout.n_groups);
  *out = h;
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_set_group(fmm_tucker_t h, int32_t group, int32_t alpha, int32_t r_theta,
                                           int32_t r_phi, int32_t r_beta, const double* core, const double* u_theta,
                                           const double* u_phi, const double* u_beta) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  const Layout& L = h->layout;
  if (group < 0 || group >= L.n_groups) return fail(FMM_ERR_ARG, "group %d out of range", group);
  if (alpha != 0 && alpha != 1) return fail(FMM_ERR_ARG, "alpha must be 0 or 1");
  const int nb = L.nb(group);
  if (r_theta < 1 || r_theta > L.n_theta || r_phi < 1 || r_phi > L.n_phi || r_beta < 1 || r_beta > nb)
    return fail(FMM_ERR_SHAPE, "ranks (%d, %d, %d) outside [1, (%d, %d, %d)]", r_theta, r_phi, r_beta, L.n_theta,
                L.n_phi, nb);
  if (!core || !u_theta || !u_phi || !u_beta) return fail(FMM_ERR_ARG, "factor pointers must be non-NULL");
  TensorFactors tf;
  tf.rt = r_theta;
  tf.rp = r_phi;
  tf.rb = r_beta;
  auto take = [](const double* p, size_t n, std::vector<cd>& v) {
    v.resize(n);
    for (size_t i = 0; i < n; ++i) v[i] = cd(p[2 * i], p[2 * i + 1]);
  };
  take(core, (size_t)r_theta * r_phi * r_beta, tf.core);
  take(u_theta, (size_t)L.n_theta * r_theta, tf.ut);
  take(u_phi, (size_t)L.n_phi * r_phi, tf.up);
  take(u_beta, (size_t)nb * r_beta, tf.ub);
  for (auto* v : {&tf.core, &tf.ut, &tf.up, &tf.ub})
    for (const cd& z : *v)
      if (!std::isfinite(z.real()) || !std::isfinite(z.imag()))
        return fail(FMM_ERR_NUMERIC, "non-finite factor entry in group %d polarisation %d", group, alpha);
  // identity angular factors (the truncated-SVD method): no angular products
  auto is_eye = [](const std::vector<cd>& m, int n) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (m[(size_t)i * n + j] != cd(i == j ? 1.0 : 0.0, 0.0)) return false;
    return true;
  };
  tf.ident = r_theta == L.n_theta && r_phi == L.n_phi && is_eye(tf.ut, r_theta) && is_eye(tf.up, r_phi);
  h->t[2 * (size_t)group + alpha] = std::move(tf);
  drop_graph(h);
  for (auto& s : h->slot) {  // uploads are stale now
    s.ready = false;
    mrhs_release(s);
    s.tuned.clear();
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_set_box_grid(fmm_tucker_t h, int32_t kx, int32_t ky, int32_t kz,
                                              const int64_t* box_of_group) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  const int G = h->layout.n_groups;
  std::vector<int64_t> box;
  int64_t K = 0;
  if (kx == 0 && ky == 0 && kz == 0 && box_of_group == nullptr) {
    // back to the group-compact layout
  } else {
    if (kx < 1 || ky < 1 || kz < 1) return fail(FMM_ERR_ARG, "box grid sizes must be >= 1 (or all 0 to clear)");
    if (!box_of_group) return fail(FMM_ERR_ARG, "box_of_group is NULL");
    K = (int64_t)kx * ky * kz;
    if (K > (int64_t)1 << 30) return fail(FMM_ERR_SIZE, "box grid of %lld boxes exceeds 2^30", (long long)K);
    if (K < G) return fail(FMM_ERR_SHAPE, "%lld boxes cannot hold %d groups", (long long)K, G);
    std::vector<char> used((size_t)K, 0);
    box.assign(box_of_group, box_of_group + G);
    for (int g = 0; g < G; ++g) {
      if (box[g] < 0 || box[g] >= K) return fail(FMM_ERR_ARG, "box of group %d out of range", g);
      if (used[(size_t)box[g]]) return fail(FMM_ERR_ARG, "box %lld holds two groups", (long long)box[g]);
      used[(size_t)box[g]] = 1;
    }
  }
  h->n_boxes = K;
  h->box_dims[0] = K ? kx : 0;
  h->box_dims[1] = K ? ky : 0;
  h->box_dims[2] = K ? kz : 0;
  h->box = std::move(box);
  drop_graph(h);
  for (auto& s : h->slot) {  // item rows and zero lists live in the arenas: upload again
    s.ready = false;
    mrhs_release(s);
    s.tuned.clear();
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_layout(fmm_tucker_t h, fmm_layout* out) {
  clear_error();
  if (!h || !out) return fail(FMM_ERR_ARG, "handle and out must be non-NULL");
  out->n_theta = h->layout.n_theta;
  out->n_phi = h->layout.n_phi;
  out->n_groups = h->layout.n_groups;
  out->reserved = 0;
  out->offsets = h->layout.offsets.data();
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_ranks(fmm_tucker_t h, int32_t* ranks) {
  clear_error();
  if (!h || !ranks) return fail(FMM_ERR_ARG, "handle and ranks must be non-NULL");
  for (size_t i = 0; i < h->t.size(); ++i) {
    ranks[3 * i + 0] = h->t[i].rt;
    ranks[3 * i + 1] = h->t[i].rp;
    ranks[3 * i + 2] = h->t[i].rb;
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_export(fmm_tucker_t h, int32_t group, int32_t alpha, fmm_prec as_stored,
                                        double* core, double* u_theta, double* u_phi, double* u_beta) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  if (group < 0 || group >= h->layout.n_groups || (alpha != 0 && alpha != 1))
    return fail(FMM_ERR_ARG, "group/alpha out of range");
  if (!prec_valid(as_stored)) return fail(FMM_ERR_ARG, "bad precision %d", (int)as_stored);
  const TensorFactors& tf = h->t[2 * (size_t)group + alpha];
  if (!tf.set()) return fail(FMM_ERR_STATE, "factors of group %d polarisation %d are not set", group, alpha);
  // the complex64 arena (every precision but FMM_C128) holds each part rounded to the
  // nearest float (pack_tensor)
  auto stored = [as_stored](double v) -> double { return as_stored == FMM_C128 ? v : (double)(float)v; };
  auto give = [&stored](const std::vector<cd>& v, double* p) {
    if (!p) return;
    for (size_t i = 0; i < v.size(); ++i) {
      p[2 * i] = stored(v[i].real());
      p[2 * i + 1] = stored(v[i].imag());
    }
  };
  give(tf.core, core);
  give(tf.ut, u_theta);
  give(tf.up, u_phi);
  give(tf.ub, u_beta);
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_storage_bytes(fmm_tucker_t h, fmm_prec prec, size_t* factor_bytes,
                                               size_t* arena_bytes) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  if (!prec_valid(prec)) return fail(FMM_ERR_ARG, "bad precision %d", (int)prec);
  ArenaPlan P;
  fmm_status st = plan_arena(h, prec, &P);
  if (st != FMM_OK) return st;
  if (factor_bytes) *factor_bytes = P.factor_bytes_paper;
  if (arena_bytes) *arena_bytes = P.total_bytes;
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_upload(fmm_tucker_t h, fmm_prec prec, void* arena, size_t bytes, void* stream) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  if (!prec_valid(prec)) return fail(FMM_ERR_ARG, "bad precision %d", (int)prec);
  fmm_status st = check_vec(arena, 256, "arena");
  if (st != FMM_OK) return st;
  ArenaPlan P;
  st = plan_arena(h, prec, &P);
  if (st != FMM_OK) return st;
  if (bytes < P.total_bytes) return fail(FMM_ERR_SIZE, "arena has %zu bytes, needs %zu", bytes, P.total_bytes);
  if (!have_device()) return FMM_ERR_DEVICE;
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));

  // host image of the whole arena
  std::vector<char> img(P.total_bytes, 0);
  char* p = img.data();
  std::memcpy(p, P.items.data(), P.items.size() * sizeof(TuckItem));
  p += P.items.size() * sizeof(TuckItem);
  const size_t units_off = (size_t)(p - img.data());
  std::memcpy(p, P.units.data(), P.units.size() * sizeof(TuckUnit));
  p += P.units.size() * sizeof(TuckUnit);
  const size_t splits_off = (size_t)(p - img.data());
  if (!P.splits.empty()) std::memcpy(p, P.splits.data(), P.splits.size() * sizeof(TuckSplit));
  p += P.splits.size() * sizeof(TuckSplit);
  const size_t order_off = (size_t)(p - img.data());
  std::memcpy(p, P.order.data(), P.order.size() * sizeof(int32_t));
  p += P.order.size() * sizeof(int32_t);
  const size_t pass_off = (size_t)(p - img.data());
  std::memcpy(p, P.pass.data(), P.pass.size() * sizeof(int32_t));
  p += P.pass.size() * sizeof(int32_t);
  const size_t zero_off = (size_t)(p - img.data());
  if (!P.zero_rows.empty()) std::memcpy(p, P.zero_rows.data(), P.zero_rows.size() * sizeof(int32_t));
  char* fac = img.data() + P.header_bytes;
  const size_t n_t = P.items.size();
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < nthreads; ++w)
    pool.emplace_back([&, w]() {
      for (size_t i = w; i < n_t; i += nthreads) {
        if (prec == FMM_C128)
          pack_tensor<double>(h->layout, h->t[i], P.items[i], reinterpret_cast<double*>(fac));
        else
          pack_tensor<float>(h->layout, h->t[i], P.items[i], reinterpret_cast<float*>(fac));
      }
    });
  for (auto& th : pool) th.join();

  hipStream_t s = static_cast<hipStream_t>(stream);
  TFMM_HIP(hipMemcpyAsync(arena, img.data(), img.size(), hipMemcpyHostToDevice, s));
  TFMM_HIP(hipStreamSynchronize(s));
  int lds_lim = 0;
  TFMM_HIP(hipDeviceGetAttribute(&lds_lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));

  PrecSlot& sl = h->slot[prec];
  drop_graph(h);
  mrhs_release(sl);
  sl.tuned.clear();
  sl.items = P.items;
  {
    // workgroup size of the streaming kernels from the mean streamed elements per item:
    // small items leave most of a large workgroup idle
    double c = 0.0;
    for (const TuckUnit& u : P.units) c += item_cost(P.items[u.item]) * (u.b1 - u.b0) / P.items[u.item].rb;
    c /= std::max<size_t>(1, P.units.size());
    // (measured on MI355X, FP32 pass.  Angular operands read from memory: mean 12k
    // elements runs best at 64 threads, 50k at 128, 258k at 256, 1.7M at 512.  Staged
    // in LDS, the shorter angular phases favour wider workgroups: 12k and 50k at 128,
    // 258k at 512.)
    const int t_plain = c >= 1.5e6 ? 512 : (c >= 1e5 ? 256 : (c >= 3e4 ? 128 : 64));
    const int t_staged = c >= 1e5 ? 512 : (c >= 5e3 ? 128 : 64);
    // Staging the angular operands (and G) in LDS shortens the angular phases but
    // takes LDS from the resident workgroups: it pays while a CU still holds
    // kStageMinWaves wavefronts (FP64 at 1-lambda boxes, 4 wavefronts staged, ran
    // 1.24 ms unstaged and 1.59 ms staged; every layout with 8 or more gained).
    TuckMax ms = P.mx;
    ms.stage = 1;
    const size_t staged = prec == FMM_C128 ? tucker_lds_bytes<double>(ms) : tucker_lds_bytes<float>(ms);
    const int waves = staged > kCuLds ? 0 : (int)(kCuLds / staged) * (t_staged / 64);
    P.mx.stage = staged <= (size_t)lds_lim && waves >= kStageMinWaves ? 1 : 0;
    if (const char* env = std::getenv("TUCKFMM_STAGE_ANGULAR")) P.mx.stage = P.mx.stage && std::atoi(env) != 0;
    sl.threads = P.mx.stage ? t_staged : t_plain;
    if (const char* env = std::getenv("TUCKFMM_STREAM_THREADS")) {
      const int v = std::atoi(env);
      if (v == 64 || v == 128 || v == 256 || v == 512) sl.threads = v;
    }
  }
  sl.streams = (prec == FMM_C128 ? tucker_lds_bytes<double>(P.mx) : tucker_lds_bytes<float>(P.mx)) <=
               (size_t)lds_lim;
  sl.ready = true;
  sl.arena = static_cast<char*>(arena);
  sl.bytes = bytes;
  sl.device = dev;
  TuckPlan& pl = sl.plan;
  pl.items = reinterpret_cast<const TuckItem*>(sl.arena);
  pl.order = reinterpret_cast<const int32_t*>(sl.arena + order_off);
  pl.pass_list = reinterpret_cast<const int32_t*>(sl.arena + pass_off);
  pl.zero_rows = P.zero_rows.empty() ? nullptr : reinterpret_cast<const int32_t*>(sl.arena + zero_off);
  pl.n_zero_rows = (int)P.zero_rows.size();
  pl.units = reinterpret_cast<const TuckUnit*>(sl.arena + units_off);
  pl.splits = P.splits.empty() ? nullptr : reinterpret_cast<const TuckSplit*>(sl.arena + splits_off);
  pl.n_units = (int)P.units.size();
  pl.n_splits = (int)P.splits.size();
  pl.part_stride = P.part_stride;
  pl.part = nullptr;
  pl.next = sl.next;
  pl.n_items = (int)P.items.size();
  pl.n_basis = h->layout.n_basis();
  pl.factors = sl.arena + P.header_bytes;
  pl.mx = P.mx;
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_aggregate(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                           void* stream) {
  clear_error();
  PrecSlot* s = nullptr;
  fmm_status st = ready_slot(h, prec, nrhs, &s);
  if (st != FMM_OK) return st;
  const size_t es = elem_bytes(prec);
  if ((st = check_vec(x, es, "x")) != FMM_OK || (st = check_vec(F, es, "F")) != FMM_OK) return st;
  return run_stage(h, *s, prec, nrhs, 0, x, F, nullptr, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" fmm_status fmm_tucker_disaggregate(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* G, void* V,
                                              void* stream) {
  clear_error();
  PrecSlot* s = nullptr;
  fmm_status st = ready_slot(h, prec, nrhs, &s);
  if (st != FMM_OK) return st;
  const size_t es = elem_bytes(prec);
  if ((st = check_vec(G, es, "G")) != FMM_OK || (st = check_vec(V, es, "V")) != FMM_OK) return st;
  return run_stage(h, *s, prec, nrhs, 1, nullptr, nullptr, G, V, static_cast<hipStream_t>(stream));
}

namespace {
fmm_status pass_checks(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F, const void* G, void* V,
                       PrecSlot** s) {
  fmm_status st = ready_slot(h, prec, nrhs, s);
  if (st != FMM_OK) return st;
  const size_t es = elem_bytes(prec);
  if ((st = check_vec(x, es, "x")) != FMM_OK || (st = check_vec(F, es, "F")) != FMM_OK ||
      (st = check_vec(G, es, "G")) != FMM_OK || (st = check_vec(V, es, "V")) != FMM_OK)
    return st;
  return FMM_OK;
}
}  // namespace

extern "C" fmm_status fmm_tucker_pass(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                      const void* G, void* V, void* stream) {
  clear_error();
  PrecSlot* s = nullptr;
  fmm_status st = pass_checks(h, prec, nrhs, x, F, G, V, &s);
  if (st != FMM_OK) return st;
  return run_stage(h, *s, prec, nrhs, 2, x, F, G, V, static_cast<hipStream_t>(stream));
}

fmm_status tuckfmm::noalloc_pass(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F, const void* G,
                                 void* V, hipStream_t hs, void* scratch, size_t scratch_bytes) {
  PrecSlot* s = nullptr;
  fmm_status st = pass_checks(h, prec, nrhs, x, F, G, V, &s);
  if (st != FMM_OK) return st;
  if (prec_is_split(prec))
    return fail(FMM_ERR_UNSUPPORTED, "the bf16 split precisions run on the matrix-core path, whose tables the "
                                     "library allocates; the allocation-free pass takes FMM_C128 or FMM_C64");
  if (prec == FMM_C128 && !s->streams)
    return fail(FMM_ERR_UNSUPPORTED, "this layout's FP64 items do not fit the streaming kernels' LDS");
  Route r;
  if ((st = route_of(*s, prec, nrhs, &r)) != FMM_OK) return st;
  const Layout& L = h->layout;
  // the slot's own counter and partial-sum buffer stay untouched: the scratch holds the
  // pass kernel's work counter in its first 256 bytes, then the partial sums
  TuckPlan pl = s->plan;
  pl.next = static_cast<int32_t*>(scratch);
  pl.part = nullptr;
  if (pl.n_splits > 0) {
    const size_t need = (size_t)pl.part_stride * (size_t)nrhs * elem_bytes(prec);
    if (need > scratch_bytes - 256)
      return fail(FMM_ERR_SIZE, "the split items' partial sums need %zu bytes for nrhs = %d, the static scratch "
                                "holds %zu after the work counter", need, nrhs, scratch_bytes - 256);
    pl.part = static_cast<char*>(scratch) + 256;
  }
  if (s->plan.n_zero_rows > 0)
    TFMM_HIP(launch_zero_rows(elem_bytes(prec), F, pl.zero_rows, pl.n_zero_rows, (int64_t)L.ndir() * nrhs, hs));
  if (prec == FMM_C128) {
    if ((st = lds_check(tucker_lds_bytes<double>(pl.mx))) != FMM_OK) return st;
    TFMM_HIP(launch_tucker_pass<double>(pl, r.threads, L.n_theta, L.n_phi, nrhs, x, F, G, V, hs));
  } else {
    if ((st = lds_check(tucker_lds_bytes<float>(pl.mx))) != FMM_OK) return st;
    TFMM_HIP(launch_tucker_pass<float>(pl, r.threads, L.n_theta, L.n_phi, nrhs, x, F, G, V, hs));
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_graph_capture(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                        const void* G, void* V, void* stream) {
  clear_error();
  PrecSlot* s = nullptr;
  fmm_status st = pass_checks(h, prec, nrhs, x, F, G, V, &s);
  if (st != FMM_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (hs == nullptr) return fail(FMM_ERR_ARG, "graph capture needs a non-default stream");
  drop_graph(h);
  // build the multi-RHS tables now: nothing may allocate or copy inside the capture
  Route r;
  if ((st = route_of(*s, prec, nrhs, &r)) != FMM_OK) return st;
  if (r.mfma) {
    MrhsPlan* mp = nullptr;
    if ((st = mrhs_get(*s, elem_bytes(prec), h->layout, nrhs, r.tile_steps, r.rhs_chunk, r.order, &mp)) != FMM_OK)
      return st;
  } else if ((st = ensure_part(h, *s, prec, nrhs)) != FMM_OK) {
    return st;
  }
  TFMM_HIP(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal));
  fmm_status d = run_stage(h, *s, prec, nrhs, 2, x, F, G, V, hs);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(hs, &graph);
  if (d != FMM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return d;
  }
  if (e != hipSuccess) return fail(FMM_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  h->graph = graph;
  TFMM_HIP(hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0));
  return FMM_OK;
}

namespace {

// Key of a tuning result: the layout's shapes (groups, ranks, identity flags, box
// grid) hashed with FNV-1a, the precision, nrhs and the hash of the kernel sources
// this library was built from.  Factor values do not change the timings.
uint64_t layout_hash(const fmm_tucker_s* h) {
  uint64_t v = 1469598103934665603ull;
  auto mix = [&v](int64_t x) {
    for (int b = 0; b < 8; ++b) {
      v ^= (uint64_t)((x >> (8 * b)) & 0xff);
      v *= 1099511628211ull;
    }
  };
  mix(h->layout.n_theta);
  mix(h->layout.n_phi);
  mix(h->layout.n_groups);
  for (int64_t o : h->layout.offsets) mix(o);
  for (const TensorFactors& t : h->t) {
    mix(t.rt);
    mix(t.rp);
    mix(t.rb);
    mix(t.ident ? 1 : 0);
  }
  mix(h->n_boxes);
  for (int64_t b : h->box) mix(b);
  return v;
}

// Checks a configuration for (prec, nrhs) on this slot.
fmm_status check_choice(const PrecSlot& s, fmm_prec prec, int nrhs, const TuneChoice& c) {
  if (c.path == 0) {
    if (prec_is_split(prec)) return fail(FMM_ERR_UNSUPPORTED, "the bf16 split precisions have no streaming kernels");
    if (prec == FMM_C128 && !s.streams)
      return fail(FMM_ERR_UNSUPPORTED, "this layout's FP64 items do not fit the streaming kernels' LDS");
    if (c.threads != 64 && c.threads != 128 && c.threads != 256 && c.threads != 512)
      return fail(FMM_ERR_ARG, "threads must be 64, 128, 256 or 512");
  } else if (c.path == 1) {
    if (!mfma_allows(prec, nrhs)) return fail(FMM_ERR_UNSUPPORTED, "the bf16 split precisions need an even nrhs");
    if (c.tile_steps < 1 || c.tile_steps > 4096) return fail(FMM_ERR_ARG, "tile_steps must be in [1, 4096]");
    if (c.rhs_chunk < 1) return fail(FMM_ERR_ARG, "rhs_chunk must be >= 1");
    if (prec_is_split(prec) && c.rhs_chunk % 2 && c.rhs_chunk < nrhs)
      return fail(FMM_ERR_ARG, "the bf16 split precisions need an even rhs_chunk");
    if (c.order < 0 || c.order > 2) return fail(FMM_ERR_ARG, "order must be 0, 1 or 2");
  } else {
    return fail(FMM_ERR_ARG, "path must be 0 or 1");
  }
  return FMM_OK;
}

void put_choice(PrecSlot& s, const TuneChoice& c) {
  s.tuned.erase(std::remove_if(s.tuned.begin(), s.tuned.end(), [&](const TuneChoice& t) { return t.nrhs == c.nrhs; }),
                s.tuned.end());
  s.tuned.push_back(c);
}

void fill_result(const TuneChoice& c, int nrhs, float ms, int from_cache, fmm_tune_result* out) {
  if (!out) return;
  out->path = c.path;
  out->tile_steps = c.path == 1 ? c.tile_steps : 0;
  out->rhs_chunk = c.path == 1 ? std::min(c.rhs_chunk, nrhs) : 0;
  out->threads = c.path == 0 ? c.threads : 0;
  out->ms = ms;
  out->order = c.path == 1 ? c.order : 0;
  out->from_cache = from_cache;
}

// Tuning cache (file named by TUCKFMM_TUNE_CACHE): one line per result,
//   tuckfmm-tune <layout hash> <source hash> <prec> <nrhs> <path> <tile_steps> <rhs_chunk> <threads> <order> <ms>
bool cache_lookup(const char* path, uint64_t key, fmm_prec prec, int nrhs, TuneChoice* c, float* ms) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char tag[32], src[64];
    unsigned long long k = 0;
    int p = 0, n = 0, pa = 0, ts = 0, rc = 0, th = 0, od = 0;
    float t = 0.f;
    if (std::sscanf(line, "%31s %llx %63s %d %d %d %d %d %d %d %f", tag, &k, src, &p, &n, &pa, &ts, &rc, &th, &od,
                    &t) != 11)
      continue;
    if (std::strcmp(tag, "tuckfmm-tune") || k != key || std::strcmp(src, TUCKFMM_SOURCE_SHA) || p != (int)prec ||
        n != nrhs)
      continue;
    *c = TuneChoice{nrhs, pa, ts, rc, th, od};
    *ms = t;
    found = true;  // the last matching line wins
  }
  std::fclose(f);
  return found;
}

void cache_append(const char* path, uint64_t key, fmm_prec prec, int nrhs, const TuneChoice& c, float ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // the cache is an optimisation: an unwritable file is ignored
  std::fprintf(f, "tuckfmm-tune %016llx %s %d %d %d %d %d %d %d %.6g\n", (unsigned long long)key, TUCKFMM_SOURCE_SHA,
               (int)prec, nrhs, c.path, c.tile_steps, c.rhs_chunk, c.threads, c.order, ms);
  std::fclose(f);
}

}  // namespace

extern "C" fmm_status fmm_tucker_set_tuned(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const fmm_tune_result* choice) {
  clear_error();
  if (!h || !choice) return fail(FMM_ERR_ARG, "handle and choice must be non-NULL");
  if (!prec_valid(prec)) return fail(FMM_ERR_ARG, "bad precision %d", (int)prec);
  if (nrhs < 1 || nrhs > 65535) return fail(FMM_ERR_ARG, "nrhs must be in [1, 65535]");
  PrecSlot& s = h->slot[prec];
  if (!s.ready) return fail(FMM_ERR_STATE, "precision %d has not been uploaded", (int)prec);
  const TuneChoice c{nrhs, choice->path, choice->tile_steps, choice->rhs_chunk, choice->threads, choice->order};
  fmm_status st = check_choice(s, prec, nrhs, c);
  if (st != FMM_OK) return st;
  drop_graph(h);
  put_choice(s, c);
  return FMM_OK;
}

extern "C" fmm_status fmm_tucker_tune(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                      const void* G, void* V, void* stream, fmm_tune_result* out) {
  clear_error();
  PrecSlot* s = nullptr;
  fmm_status st = pass_checks(h, prec, nrhs, x, F, G, V, &s);
  if (st != FMM_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  TFMM_HIP(hipStreamIsCapturing(hs, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(FMM_ERR_STATE, "cannot tune inside a stream capture");
  const char* cache = std::getenv("TUCKFMM_TUNE_CACHE");
  if (cache && !*cache) cache = nullptr;
  const uint64_t key = layout_hash(h);
  if (cache) {
    TuneChoice c;
    float ms = 0.f;
    if (cache_lookup(cache, key, prec, nrhs, &c, &ms) && check_choice(*s, prec, nrhs, c) == FMM_OK) {
      drop_graph(h);
      put_choice(*s, c);
      fill_result(c, nrhs, ms, 1, out);
      return FMM_OK;
    }
    clear_error();
  }
  // candidates: the streaming kernels (FP64, FP32; FP64 only where its items fit their
  // LDS) and the matrix-core products with several tile sizes, right-hand-side chunks
  // and angular contraction orders (any nrhs; an even one for the bf16 split
  // precisions)
  std::vector<TuneChoice> cand;
  if (!prec_is_split(prec) && (prec != FMM_C128 || s->streams))
    for (int nt : {64, 128, 256, 512}) cand.push_back(TuneChoice{nrhs, 0, 0, 0, nt, 0});
  if (mfma_allows(prec, nrhs)) {
    std::vector<int> chunks{std::min<int>(nrhs, kMrhsDefaultChunk)};
    if (nrhs > 2 * kMrhsDefaultChunk) chunks.push_back(2 * kMrhsDefaultChunk);
    if (nrhs >= kMrhsDefaultChunk) chunks.push_back(kMrhsDefaultChunk / 2);
    for (int od : {0, 1, 2})
      for (int ts : {8, 16, 32, 64})
        for (int rc : chunks) cand.push_back(TuneChoice{nrhs, 1, ts, rc, 0, od});
  }
  if (cand.empty()) return fail(FMM_ERR_UNSUPPORTED, "no kernels for precision %d with nrhs %d", (int)prec, nrhs);
  // tables that existed before the call stay; a candidate's new tables are freed as soon
  // as a faster one is found, so at most two candidates' scratch is held at a time
  std::vector<const MrhsPlan*> before;
  for (const MrhsPlan& p : s->mrhs) before.push_back(&p);
  auto is_before = [&](const MrhsPlan* p) { return std::find(before.begin(), before.end(), p) != before.end(); };
  auto plan_of = [&](const TuneChoice& c) -> MrhsPlan* {
    if (c.path != 1) return nullptr;
    for (MrhsPlan& p : s->mrhs)
      if (p.nrhs == nrhs && p.tile_steps == c.tile_steps && p.rhs_chunk == std::min(c.rhs_chunk, nrhs) &&
          p.order == c.order)
        return &p;
    return nullptr;
  };
  auto release = [&](MrhsPlan* p) {
    if (!p || is_before(p)) return;
    for (auto it = s->mrhs.begin(); it != s->mrhs.end(); ++it)
      if (&*it == p) {
        mrhs_free(*it);
        s->mrhs.erase(it);
        return;
      }
  };
  const std::vector<TuneChoice> saved = s->tuned;
  drop_graph(h);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TFMM_HIP(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(FMM_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(he));
  }
  const int reps = 3;
  float best = -1.f;
  TuneChoice win{};
  for (const TuneChoice& c : cand) {
    s->tuned.assign(1, c);
    st = run_stage(h, *s, prec, nrhs, 2, x, F, G, V, hs);  // warm-up (builds the tables)
    if (st == FMM_ERR_UNSUPPORTED) {  // a candidate this layout cannot take
      st = FMM_OK;
      clear_error();
      continue;
    }
    if (st != FMM_OK) break;
    he = hipEventRecord(e0, hs);
    for (int i = 0; i < reps && st == FMM_OK; ++i) st = run_stage(h, *s, prec, nrhs, 2, x, F, G, V, hs);
    if (he == hipSuccess) he = hipEventRecord(e1, hs);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (st != FMM_OK || he != hipSuccess) break;
    ms /= reps;
    if (best < 0.f || ms < best) {
      if (best >= 0.f) release(plan_of(win));
      best = ms;
      win = c;
    } else {
      release(plan_of(c));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->tuned = saved;
  if (st == FMM_OK && he != hipSuccess) st = fail(FMM_ERR_DEVICE, "tuning timer: %s", hipGetErrorString(he));
  if (st == FMM_OK && best < 0.f)
    st = fail(FMM_ERR_UNSUPPORTED, "no kernel runs precision %d with nrhs %d on this layout", (int)prec, nrhs);
  if (st != FMM_OK) {  // keep only the tables that existed before
    for (auto it = s->mrhs.begin(); it != s->mrhs.end();) {
      if (is_before(&*it)) {
        ++it;
      } else {
        mrhs_free(*it);
        it = s->mrhs.erase(it);
      }
    }
    return st;
  }
  put_choice(*s, win);
  if (cache) cache_append(cache, key, prec, nrhs, win, best);
  fill_result(win, nrhs, best, 0, out);
  return FMM_OK;
}

extern "C" fmm_status fmm_graph_launch(fmm_tucker_t h, void* stream) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  if (!h->graph_exec) return fail(FMM_ERR_STATE, "no captured graph");
  TFMM_HIP(hipGraphLaunch(h->graph_exec, static_cast<hipStream_t>(stream)));
  return FMM_OK;
}

extern "C" void fmm_tucker_destroy(fmm_tucker_t h) {
  if (!h) return;
  drop_graph(h);
  for (auto& s : h->slot) {
    mrhs_release(s);
    part_release(s);
  }
  delete h;
}

// ---------------------------------------------------------------------- dense

extern "C" fmm_status fmm_dense_create(const fmm_layout* layout, fmm_dense_t* out) {
  clear_error();
  if (!out) return fail(FMM_ERR_ARG, "out is NULL");
  *out = nullptr;
  auto* d = new fmm_dense_s();
  fmm_status st = copy_layout(layout, &d->layout);
  if (st != FMM_OK) {
    delete d;
    return st;
  }
  if (!have_device()) {
    delete d;
    return FMM_ERR_DEVICE;
  }
  const int G = d->layout.n_groups;
  std::vector<DenseGroup> grp(G);
  for (int g = 0; g < G; ++g) grp[g] = DenseGroup{d->layout.offsets[g], d->layout.nb(g), 0};
  // Row blocks of the multi-RHS disaggregation.  Workgroups go to the eight XCDs
  // round-robin by index; the list gives XCD x the x-th eighth of the blocks in group
  // order (position 8 j + x holds block x * per + j), so that the few groups an XCD
  // works on at a time keep their G in its L2.
  std::vector<DenseBlock> nat;
  for (int g = 0; g < G; ++g)
    for (int i = 0; i < d->layout.nb(g); i += kDenseBlockRows)
      nat.push_back(DenseBlock{d->layout.offsets[g] + i, std::min(kDenseBlockRows, d->layout.nb(g) - i), g});
  std::vector<DenseBlock> blk;
  blk.reserve(nat.size());
  const size_t per = (nat.size() + 7) / 8;
  for (size_t j = 0; j < per; ++j)
    for (size_t x = 0; x < 8; ++x)
      if (x * per + j < nat.size()) blk.push_back(nat[x * per + j]);
  d->n_blocks = (int)blk.size();
  hipError_t e = hipGetDevice(&d->device);
  if (e == hipSuccess && G > 0) e = hipMalloc(&d->d_groups, sizeof(DenseGroup) * G);
  if (e == hipSuccess) e = hipMalloc(&d->d_offsets, sizeof(int64_t) * (G + 1));
  if (e == hipSuccess && !blk.empty()) e = hipMalloc(&d->d_blocks, sizeof(DenseBlock) * blk.size());
  if (e == hipSuccess && G > 0)
    e = hipMemcpy(d->d_groups, grp.data(), sizeof(DenseGroup) * G, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d->d_offsets, d->layout.offsets.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && !blk.empty())
    e = hipMemcpy(d->d_blocks, blk.data(), sizeof(DenseBlock) * blk.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    fmm_dense_destroy(d);
    return fail(FMM_ERR_DEVICE, "dense plan upload: %s", hipGetErrorString(e));
  }
  *out = d;
  return FMM_OK;
}

namespace {
fmm_status dense_common(fmm_dense_t d, fmm_prec prec, const void* A, int32_t nrhs, const void* in, void* out) {
  if (!d) return fail(FMM_ERR_ARG, "plan is NULL");
  if (!prec_valid(prec)) return fail(FMM_ERR_ARG, "bad precision %d", (int)prec);
  if (prec != FMM_C128 && prec != FMM_C64)
    return fail(FMM_ERR_UNSUPPORTED, "the dense path supports FMM_C128 and FMM_C64 only");
  if (nrhs < 1 || nrhs > 65535) return fail(FMM_ERR_ARG, "nrhs must be in [1, 65535]");
  const size_t es = elem_bytes(prec);
  fmm_status st;
  if ((st = check_vec(A, es, "farfield")) != FMM_OK || (st = check_vec(in, es, "input")) != FMM_OK ||
      (st = check_vec(out, es, "output")) != FMM_OK)
    return st;
  if (!have_device()) return FMM_ERR_DEVICE;
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));
  if (dev != d->device) return fail(FMM_ERR_STATE, "current device differs from the plan's device");
  return FMM_OK;
}
}  // namespace

extern "C" fmm_status fmm_dense_aggregate(fmm_dense_t d, fmm_prec prec, const void* farfield, int32_t nrhs,
                                          const void* x, void* F, void* stream) {
  clear_error();
  fmm_status st = dense_common(d, prec, farfield, nrhs, x, F);
  if (st != FMM_OK) return st;
  const int ncols = 2 * d->layout.ndir();
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (prec == FMM_C128)
    TFMM_HIP(launch_dense_agg<double>(farfield, d->d_groups, d->layout.n_groups, ncols, nrhs, x, F, hs));
  else
    TFMM_HIP(launch_dense_agg<float>(farfield, d->d_groups, d->layout.n_groups, ncols, nrhs, x, F, hs));
  return FMM_OK;
}

extern "C" fmm_status fmm_dense_disaggregate(fmm_dense_t d, fmm_prec prec, const void* farfield, int32_t nrhs,
                                             const void* G, void* V, void* stream) {
  clear_error();
  fmm_status st = dense_common(d, prec, farfield, nrhs, G, V);
  if (st != FMM_OK) return st;
  const int ncols = 2 * d->layout.ndir();
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (prec == FMM_C128)
    TFMM_HIP(launch_dense_disagg<double>(farfield, d->d_offsets, d->layout.n_groups, d->layout.n_basis(),
                                         d->d_blocks, d->n_blocks, ncols, nrhs, G, V, hs));
  else
    TFMM_HIP(launch_dense_disagg<float>(farfield, d->d_offsets, d->layout.n_groups, d->layout.n_basis(),
                                        d->d_blocks, d->n_blocks, ncols, nrhs, G, V, hs));
  return FMM_OK;
}

extern "C" void fmm_dense_destroy(fmm_dense_t d) {
  if (!d) return;
  if (d->d_groups) (void)hipFree(d->d_groups);
  if (d->d_offsets) (void)hipFree(d->d_offsets);
  if (d->d_blocks) (void)hipFree(d->d_blocks);
  delete d;
}
