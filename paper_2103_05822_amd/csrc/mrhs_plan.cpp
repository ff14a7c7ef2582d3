// Host-side plan of the multi-right-hand-side path.
//
// With R right-hand sides the Tucker aggregation (Section II.C, Fig. 2(b)) and
// disaggregation (Fig. 3(b)) of one (group, polarisation) item are chains of four
// complex matrix products.  For a chunk of rc right-hand sides, with Q = r_theta r_phi
// and the factor layouts of the arena (U^beta^T [r_beta][ld_ub], core [r_beta][ld_c]
// with column q = a r_phi + c, U^theta [n_theta][r_theta], U^phi [n_phi][r_phi]):
//
//   aggregation                                    disaggregation (W = conj(V))
//   1  Y  [r_beta][rc]  = U^beta^T x_g              1  theta or phi contraction of conj(G)
//   2  T  [Q][rc]       = core^T Y                  2  the other angular contraction -> S2 [Q][rc]
//   3  one angular product on T                     3  s3 [r_beta][rc] = core S2
//   4  the other one, written into F                4  V_g += conj(U^beta s3)
//
// The angular order is the item's cheaper one (theta_first); the disaggregation runs
// the adjoint chain in reverse order, which has the same cost.  Launch j of a stage
// computes product j of every item (one grouped GEMM); a pass merges launch j of both
// stages.  The two polarisations of a group add into V with one atomic add each onto
// zero, so V does not depend on the order of the adds.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "internal.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

constexpr int kTileM = 64, kTileN = 64, kStepK = 16;  // tile shape of the grouped GEMM kernel

int64_t up32(int64_t n) { return (n + 31) / 32 * 32; }  // complex elements, 256-byte blocks
size_t align256(size_t v) { return (v + 255) / 256 * 256; }

CGemm make_gemm(int32_t M, int32_t N, int32_t K, int64_t a, int32_t abase, int32_t lda_m, int32_t lda_k, int64_t b,
                int32_t bbase, int32_t ldb_k, int32_t b_ni, int32_t b_shi, int64_t c, int32_t cbase, int32_t ldc_m,
                int32_t c_ni, int32_t c_shi, int32_t flags) {
  CGemm g{};
  g.a = a;
  g.b = b;
  g.c = c;
  g.abase = abase;
  g.bbase = bbase;
  g.cbase = cbase;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda_m = lda_m;
  g.lda_k = lda_k;
  g.ldb_k = ldb_k;
  g.b_ni = b_ni;
  g.b_shi = b_shi;
  g.ldc_m = ldc_m;
  g.c_ni = c_ni;
  g.c_shi = c_shi;
  g.flags = flags;
  return g;
}

// The eight products of one item for columns r0 .. r0 + rc - 1 of R.  sa / sd: the
// item's scratch blocks (complex offsets) of the two stages.
void item_products(const TuckItem& it, const Layout& L, int R, int r0, int rc, const int64_t sa[3],
                   const int64_t sd[3], CGemm out[8]) {
  const int nt = L.n_theta, np = L.n_phi, Q = it.rt * it.rp;
  const int64_t fo = (int64_t)it.frow * L.ndir() * R + r0;  // F / G of the item
  const int64_t xo = it.row0 * R + r0;                                        // x / V of the group
  const int32_t F_ = kBaseFactors, S_ = kBaseScratch;
  // aggregation
  out[0] = make_gemm(it.rb, rc, it.nb, it.off_ubt, F_, it.ld_ub, 1, xo, kBaseX, R, rc, 0, sa[0], S_, rc, rc, 0, 0);
  out[1] = make_gemm(Q, rc, it.rb, it.off_core, F_, 1, it.ld_c, sa[0], S_, rc, rc, 0, sa[1], S_, rc, rc, 0, 0);
  if (it.ident) {
    // truncated-SVD item (identity angular factors): F = W Y directly, s3 = W^T-side
    // product of conj(G); the angular products are empty (M = 0: no tiles)
    out[1].c = fo;
    out[1].cbase = kBaseF;
    out[1].ldc_m = R;
    out[2] = out[3] = out[4] = out[5] = CGemm{};
    out[6] = make_gemm(it.rb, rc, Q, it.off_core, F_, it.ld_c, 1, fo, kBaseG, R, rc, 0, sd[0], S_, rc, rc, 0, kConjB);
    out[7] = make_gemm(it.nb, rc, it.rb, it.off_ubt, F_, 1, it.ld_ub, sd[0], S_, rc, rc, 0, xo, kBaseV, R, rc, 0,
                       kAtomicC | kConjC);
    return;
  }
  if (it.theta_first) {
    // T3 [c][i][r] = sum_a U^theta[i][a] T[a rp + c][r];  F[i][j][r] = sum_c U^phi[j][c] T3[c][i][r]
    out[2] = make_gemm(nt, it.rp * rc, it.rt, it.off_ut, F_, it.rt, 1, sa[1], S_, it.rp * rc, it.rp * rc, 0, sa[2],
                       S_, rc, rc, nt * rc, 0);
    out[3] = make_gemm(np, nt * rc, it.rp, it.off_up, F_, it.rp, 1, sa[2], S_, nt * rc, nt * rc, 0, fo, kBaseF, R, rc,
                       np * R, 0);
  } else {
    // T3 [a][j][r] = sum_c U^phi[j][c] T[a rp + c][r];  F[i][j][r] = sum_a U^theta[i][a] T3[a][j][r]
    out[2] = make_gemm(np, it.rt * rc, it.rp, it.off_up, F_, it.rp, 1, sa[1], S_, rc, rc, it.rp * rc, sa[2], S_, rc,
                       rc, np * rc, 0);
    out[3] = make_gemm(nt, np * rc, it.rt, it.off_ut, F_, it.rt, 1, sa[2], S_, np * rc, np * rc, 0, fo, kBaseF, np * R,
                       rc, R, 0);
  }
  // disaggregation of W = conj(V): the adjoint chain on conj(G)
  if (!it.theta_first) {
    // S1 [a][j][r] = sum_i U^theta[i][a] conj G[i][j][r];  S2 [a][c][r] = sum_j U^phi[j][c] S1[a][j][r]
    out[4] = make_gemm(it.rt, np * rc, nt, it.off_ut, F_, 1, it.rt, fo, kBaseG, np * R, rc, R, sd[2], S_, np * rc,
                       np * rc, 0, kConjB);
    out[5] = make_gemm(it.rp, it.rt * rc, np, it.off_up, F_, 1, it.rp, sd[2], S_, rc, rc, np * rc, sd[1], S_, rc, rc,
                       it.rp * rc, 0);
  } else {
    // S1 [i][c][r] = sum_j U^phi[j][c] conj G[i][j][r];  S2 [a][c][r] = sum_i U^theta[i][a] S1[i][c][r]
    out[4] = make_gemm(it.rp, nt * rc, np, it.off_up, F_, 1, it.rp, fo, kBaseG, R, rc, np * R, sd[2], S_, rc, rc,
                       it.rp * rc, kConjB);
    out[5] = make_gemm(it.rt, it.rp * rc, nt, it.off_ut, F_, 1, it.rt, sd[2], S_, it.rp * rc, it.rp * rc, 0, sd[1], S_,
                       it.rp * rc, it.rp * rc, 0, 0);
  }
  out[6] = make_gemm(it.rb, rc, Q, it.off_core, F_, it.ld_c, 1, sd[1], S_, rc, rc, 0, sd[0], S_, rc, rc, 0, 0);
  out[7] = make_gemm(it.nb, rc, it.rb, it.off_ubt, F_, 1, it.ld_ub, sd[0], S_, rc, rc, 0, xo, kBaseV, R, rc, 0,
                     kAtomicC | kConjC);
}

struct TileCost {
  CTile t;
  int64_t cost;
  int64_t bundle;  // tiles of one product and column range: they share the B operand
};

// Work tiles of one product: 64-row blocks x groups of 64-column blocks.  A tile runs
// about tile_steps K steps; products with few column blocks keep them all in one tile
// so their (large) A operand is read once.
void tiles_of(const CGemm& g, int prob, int tile_steps, std::vector<TileCost>& out) {
  if (g.M <= 0 || g.N <= 0) return;
  const int mt = (g.M + kTileM - 1) / kTileM;
  const int nblk = (g.N + kTileN - 1) / kTileN;
  const int ks = std::max(1, (g.K + kStepK - 1) / kStepK);
  int cpt = nblk <= 4 ? nblk : std::max(1, std::min(nblk, (tile_steps + ks - 1) / ks));
  for (int b = 0; b < nblk; b += cpt) {
    const int nb = std::min(cpt, nblk - b);
    const int64_t bundle = ((int64_t)prob << 20) | b;
    for (int m = 0; m < mt; ++m) {
      TileCost tc;
      tc.t = CTile{prob, m * kTileM, b * kTileN, std::min(g.N, (b + nb) * kTileN)};
      tc.cost = (int64_t)nb * (ks + 2);
      tc.bundle = bundle;
      out.push_back(tc);
    }
  }
}

// Launch order of a tile list.  Workgroups are dispatched to the eight XCDs of the
// chip round-robin by index, and each XCD has its own L2.  Tiles that share a B
// operand (a bundle) are kept on one XCD: bundles, longest first, go to the least
// loaded of eight queues, and the list interleaves the queues so that position p
// lands on XCD p mod 8.  Each XCD then runs its bundles in longest-first order.
constexpr int kXcds = 8;

void order_tiles(std::vector<TileCost>& v) {
  if (v.empty()) return;
  std::vector<size_t> idx(v.size());
  std::iota(idx.begin(), idx.end(), 0);
  // bundles in first-appearance order with their total cost
  std::vector<int64_t> keys;
  std::vector<int64_t> cost;
  std::vector<std::vector<size_t>> members;
  {
    std::vector<size_t> by(idx);
    std::stable_sort(by.begin(), by.end(), [&](size_t a, size_t b) { return v[a].bundle < v[b].bundle; });
    for (size_t i : by) {
      if (keys.empty() || keys.back() != v[i].bundle) {
        keys.push_back(v[i].bundle);
        cost.push_back(0);
        members.emplace_back();
      }
      cost.back() += v[i].cost;
      members.back().push_back(i);
    }
  }
  std::vector<size_t> border(keys.size());
  std::iota(border.begin(), border.end(), 0);
  std::stable_sort(border.begin(), border.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<std::vector<size_t>> q(kXcds);
  std::vector<int64_t> load(kXcds, 0);
  for (size_t bi : border) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (size_t i : members[bi]) q[x].push_back(i);
    load[x] += cost[bi];
  }
  std::vector<TileCost> out;
  out.reserve(v.size());
  std::vector<size_t> head(kXcds, 0);
  while (out.size() < v.size()) {
    for (int x = 0; x < kXcds && out.size() < v.size(); ++x) {
      int src = x;
      if (head[src] == q[src].size()) {  // queue empty: take from the longest remaining one
        size_t best = 0;
        for (int y = 0; y < kXcds; ++y)
          if (q[y].size() - head[y] > best) {
            best = q[y].size() - head[y];
            src = y;
          }
      }
      out.push_back(v[q[src][head[src]++]]);
    }
  }
  v.swap(out);
}

}  // namespace

void mrhs_free(MrhsPlan& p) {
  if (p.dev) (void)hipFree(p.dev);
  p.dev = nullptr;
}

void mrhs_release(PrecSlot& s) {
  for (auto& p : s.mrhs) mrhs_free(p);
  s.mrhs.clear();
}

void mrhs_build_host(const std::vector<TuckItem>& items_in, const Layout& L, int nrhs, int tile_steps,
                     int rhs_chunk, int order, MrhsHost* out) {
  // the angular order: each item's cheaper one (order 0), or theta (1) / phi (2) first
  // for every item
  std::vector<TuckItem> items(items_in);
  if (order == 1 || order == 2)
    for (TuckItem& it : items)
      if (!it.ident) it.theta_first = order == 1 ? 1 : 0;
  const int n_items = (int)items.size();
  const int n_chunks = (nrhs + rhs_chunk - 1) / rhs_chunk;
  // scratch: per item, three blocks per stage (sized for a full chunk)
  std::vector<int64_t> sa((size_t)3 * n_items), sd((size_t)3 * n_items);
  int64_t soff = 0;
  for (int i = 0; i < n_items; ++i) {
    const TuckItem& it = items[i];
    const int64_t q = (int64_t)it.rt * it.rp;
    const int64_t t3 = it.theta_first ? (int64_t)L.n_theta * it.rp : (int64_t)it.rt * L.n_phi;
    // identity angular items keep only Y / s3 in scratch
    const int64_t sz[3] = {it.rb, it.ident ? 0 : q, it.ident ? 0 : t3};
    for (int st = 0; st < 2; ++st)
      for (int j = 0; j < 3; ++j) {
        (st ? sd : sa)[3 * i + j] = soff;
        soff += up32(sz[j] * rhs_chunk);
      }
  }
  out->scratch_elems = soff;
  out->chunks.assign(n_chunks, MrhsHostChunk{});
  for (int c = 0; c < n_chunks; ++c) {
    MrhsHostChunk& h = out->chunks[c];
    h.r0 = c * rhs_chunk;
    h.rc = std::min(rhs_chunk, nrhs - h.r0);
    h.probs.resize((size_t)8 * n_items);
    for (int i = 0; i < n_items; ++i) {
      CGemm g[8];
      item_products(items[i], L, nrhs, h.r0, h.rc, &sa[3 * i], &sd[3 * i], g);
      for (int j = 0; j < 8; ++j) h.probs[(size_t)j * n_items + i] = g[j];
    }
    for (int j = 0; j < 4; ++j) {
      std::vector<TileCost> ta, td;
      for (int i = 0; i < n_items; ++i) {
        tiles_of(h.probs[(size_t)j * n_items + i], j * n_items + i, tile_steps, ta);
        tiles_of(h.probs[(size_t)(4 + j) * n_items + i], (4 + j) * n_items + i, tile_steps, td);
      }
      std::vector<TileCost> tp(ta);
      tp.insert(tp.end(), td.begin(), td.end());
      order_tiles(ta);
      order_tiles(td);
      order_tiles(tp);
      const std::vector<TileCost>* src[3] = {&ta, &td, &tp};
      for (int k = 0; k < 3; ++k) {
        h.lists[k][j].resize(src[k]->size());
        for (size_t e = 0; e < src[k]->size(); ++e) h.lists[k][j][e] = (*src[k])[e].t;
      }
    }
  }
}

fmm_status mrhs_get(PrecSlot& s, size_t elem_bytes, const Layout& L, int nrhs, int tile_steps, int rhs_chunk,
                    int order, MrhsPlan** out) {
  if (tile_steps <= 0) tile_steps = kMrhsDefaultSteps;
  if (rhs_chunk <= 0) rhs_chunk = kMrhsDefaultChunk;
  // (any nrhs: the paired 16-byte loads read factor rows only; the callers keep the
  // bf16 split precisions to an even nrhs)
  rhs_chunk = std::min(rhs_chunk, nrhs);
  if (order < 0 || order > 2) order = 0;
  for (auto& p : s.mrhs)
    if (p.nrhs == nrhs && p.tile_steps == tile_steps && p.rhs_chunk == rhs_chunk && p.order == order) {
      *out = &p;
      return FMM_OK;
    }
  MrhsHost host;
  mrhs_build_host(s.items, L, nrhs, tile_steps, rhs_chunk, order, &host);
  const int n_chunks = (int)host.chunks.size();
  size_t table_bytes = 0;
  for (const MrhsHostChunk& h : host.chunks) {
    table_bytes += align256(h.probs.size() * sizeof(CGemm));
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 4; ++j) table_bytes += align256(h.lists[k][j].size() * sizeof(CTile));
  }
  const size_t scratch_bytes = (size_t)host.scratch_elems * elem_bytes;

  // one device allocation: tables, then scratch
  MrhsPlan p;
  p.nrhs = nrhs;
  p.rhs_chunk = rhs_chunk;
  p.tile_steps = tile_steps;
  p.order = order;
  p.dev_bytes = table_bytes + scratch_bytes;
  p.scratch_bytes = scratch_bytes;
  std::vector<char> img(table_bytes);
  size_t off = 0;
  p.chunks.resize(n_chunks);
  std::vector<size_t> prob_off(n_chunks), list_off((size_t)n_chunks * 12);
  for (int c = 0; c < n_chunks; ++c) {
    const MrhsHostChunk& h = host.chunks[c];
    prob_off[c] = off;
    std::memcpy(img.data() + off, h.probs.data(), h.probs.size() * sizeof(CGemm));
    off += align256(h.probs.size() * sizeof(CGemm));
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 4; ++j) {
        list_off[(size_t)c * 12 + k * 4 + j] = off;
        std::memcpy(img.data() + off, h.lists[k][j].data(), h.lists[k][j].size() * sizeof(CTile));
        off += align256(h.lists[k][j].size() * sizeof(CTile));
      }
  }
  TFMM_HIP(hipMalloc(&p.dev, p.dev_bytes));
  hipError_t e = hipMemcpy(p.dev, img.data(), table_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p.dev);
    return fail(FMM_ERR_DEVICE, "multi-RHS table upload: %s", hipGetErrorString(e));
  }
  p.scratch = p.dev + table_bytes;
  for (int c = 0; c < n_chunks; ++c) {
    MrhsChunk& ch = p.chunks[c];
    ch.r0 = host.chunks[c].r0;
    ch.rc = host.chunks[c].rc;
    ch.probs = reinterpret_cast<const CGemm*>(p.dev + prob_off[c]);
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 4; ++j) {
        ch.tiles[k][j] = reinterpret_cast<const CTile*>(p.dev + list_off[(size_t)c * 12 + k * 4 + j]);
        ch.n_tiles[k][j] = (int)host.chunks[c].lists[k][j].size();
      }
  }
  s.mrhs.push_back(std::move(p));
  *out = &s.mrhs.back();
  return FMM_OK;
}

fmm_status mrhs_run(const MrhsPlan& p, const PrecSlot& s, int variant, size_t elem_bytes, int stage, const void* x,
                    void* F, const void* G, void* V, hipStream_t st) {
  CGemmBases b{};
  b.p[kBaseFactors] = const_cast<void*>(s.plan.factors);
  b.p[kBaseScratch] = p.scratch;
  b.p[kBaseX] = const_cast<void*>(x);
  b.p[kBaseF] = F;
  b.p[kBaseG] = const_cast<void*>(G);
  b.p[kBaseV] = V;
  if (stage != 0) TFMM_HIP(launch_zero_cplx(elem_bytes, V, s.plan.n_basis * p.nrhs, st));
  for (const MrhsChunk& ch : p.chunks)
    for (int j = 0; j < 4; ++j) TFMM_HIP(launch_cgemm(variant, ch.probs, ch.tiles[stage][j], ch.n_tiles[stage][j], b, st));
  return FMM_OK;
}

}  // namespace tuckfmm
