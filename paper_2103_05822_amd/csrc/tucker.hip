// Tucker-format aggregation and disaggregation (Section II.C, Figs. 2(b) and 3(b)).
//
// One workgroup of NT = 64, 128, 256 or 512 threads (NT / 64 wavefronts) per
// (group, polarisation) work item, NT chosen from the mean item size.  The two large
// operands of an item -- U^beta and the core -- are streamed once from HBM with
// 16-byte coalesced loads; every intermediate stays in LDS.  Work lists are sorted by
// decreasing cost, so the hardware dispatcher hands out the largest items first
// (longest-processing-time order).  The pass kernel runs the aggregation and
// disaggregation items of all groups in one launch.  In layouts of few items, large
// items run as blocks of their r_beta rows (work units) whose partial sums a
// finishing kernel adds in block order.
//
// Aggregation of item (g, alpha), contraction order chosen per item on the host:
//   y[b]    = sum_n U^beta[n][b] x[n]          row-dot of each U^beta^T row (one
//                                              wavefront per row, lane-strided
//                                              16-byte loads, butterfly reduction)
//   t[q]    = sum_b core[b][q] y[b]            column axpy over the core rows
//                                              (one thread per column pack)
//   F[i,j]  = sum U^theta[i][a] U^phi[j][c] t[a, c]   two small LDS products
// Disaggregation of item (g, alpha), the polarisations summed as in eq. (5):
//   S[a,c]  = sum U^theta[i][a] U^phi[j][c] conj(G[i,j])   small LDS products
//   s[b]    = sum_q core[b][q] S[q]            row-dot of each core row
//   V[n]   += conj(sum_b U^beta[n][b] s[b])    column axpy over U^beta^T, added
//                                              atomically onto a zeroed V: each
//                                              entry receives exactly two additions
//                                              onto zero, which commute exactly, so
//                                              the result does not depend on which
//                                              polarisation finishes first.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

// Workgroup size NT (64, 128, 256 or 512 threads, NT / 64 wavefronts) is a template
// parameter of every phase: one workgroup per item.
constexpr int kColPacks = 2;  // column packs per thread per chunk in the axpy stages
// K values per step of the small angular products in the 64- and 128-thread kernels
// (small items): all of a step's operands are loaded before its multiply-adds.
constexpr int kSmallKUnroll = 4;

// U^beta^T and the core are read once per pass: non-temporal loads keep these
// streams from displacing x, G, V and the work tables in the caches.  Measured on
// MI355X they pay off for large items (5-7% on layouts with boxes of 2 lambda and
// more) and cost about 4% on small ones (0.5 lambda boxes), so only the 256- and
// 512-thread instantiations, which the workgroup-size rule picks for large items,
// use them.
template <typename P>
struct NtVec;
template <>
struct NtVec<float4> {
  typedef float v __attribute__((ext_vector_type(4)));
};
template <>
struct NtVec<double2> {
  typedef double v __attribute__((ext_vector_type(2)));
};
template <bool kNt, typename P>
__device__ __forceinline__ P ldnt(const P* p) {
  if (!kNt) return *p;
  const auto v = __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<P>::v*>(p));
  P o;
  __builtin_memcpy(&o, &v, sizeof(P));
  return o;
}

// LDS regions (complex elements).
// Aggregation:    r1 = x (n_beta), later t (r_theta r_phi);  r2 = y (r_beta), later
//                 the angular intermediate; with staging, sa = U^theta and U^phi^T.
// Disaggregation: s1 = angular intermediate, S (r_theta r_phi), s (r_beta); with
//                 staging, sd = conj(G) of the item and one angular factor at a time.
template <typename T>
struct Lds {
  int r1, r2, s1, s2, s3, sa, sd;
  __host__ __device__ explicit Lds(const TuckMax& mx) {
    constexpr int E = Tr<T>::E;
    r1 = round_up(max(round_up(mx.nb, E), round_up(mx.q, E)), 2);
    r2 = round_up(max(mx.rb, mx.t3), 2);
    s1 = round_up(mx.t3, 2);
    s2 = round_up(round_up(mx.q, E), 2);
    s3 = round_up(mx.rb, 2);
    sa = mx.stage ? round_up(mx.nt * mx.rt, 2) + round_up(mx.np * mx.rp, 2) : 0;
    sd = mx.stage ? round_up(mx.nt * mx.np, 2) + round_up(max(mx.nt * mx.rt, mx.np * mx.rp), 2) : 0;
  }
  __host__ __device__ size_t agg_bytes() const { return size_t(r1 + r2 + sa) * sizeof(typename Tr<T>::c); }
  __host__ __device__ size_t dis_bytes() const { return size_t(s1 + s2 + s3 + sd) * sizeof(typename Tr<T>::c); }
  __host__ __device__ size_t bytes() const { return agg_bytes() > dis_bytes() ? agg_bytes() : dis_bytes(); }
};

// Short rows (npk <= 32 packs): the wavefront splits into 64 / S segments of S lanes,
// S the smallest power of two >= npk, and each segment takes a row, four rows per
// segment in flight, so a wavefront works on 4 * 64 / S rows at once instead of four
// mostly idle ones; the segment's sum is a butterfly over its S lanes.
template <typename T, bool kNt>
__device__ __forceinline__ void wave_rowdots_short(const typename Tr<T>::c* rows, int ld, int first, int last,
                                                   int step, const typename Tr<T>::pack* vec, int npk,
                                                   typename Tr<T>::c* out, int lane) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  int S = 1;
  while (S < npk) S <<= 1;
  const int G = 64 / S;             // segments (rows) per wavefront
  const int seg = lane / S, sl = lane - seg * S;
  const bool act = sl < npk;
  const P v = act ? vec[sl] : pzero<P>();
  for (int j0 = 0; first + step * j0 < last; j0 += 4 * G) {
    P u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = first + step * (j0 + G * i + seg);
      u[i] = (act && b < last) ? ldnt<kNt>(reinterpret_cast<const P*>(rows + (int64_t)b * ld) + sl) : pzero<P>();
    }
    C a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = czero<C>();
      pdot(a[i], u[i], v);
    }
    for (int o = S >> 1; o > 0; o >>= 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i].x += __shfl_xor(a[i].x, o, 64);
        a[i].y += __shfl_xor(a[i].y, o, 64);
      }
    }
    if (sl == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int b = first + step * (j0 + G * i + seg);
        if (b < last) out[b] = a[i];
      }
    }
  }
}

// out[b] = sum_k rows[b][k] * vec[k] for b = first, first + step, ... < last, one
// wavefront per row.  Rows are 16-byte aligned with npk packs each; vec is an LDS
// pack array.  Four rows at a time, two packs per row per iteration: eight 16-byte
// loads in flight per lane.  Rows of at most 32 packs take the segmented form above.
template <typename T, bool kNt>
__device__ __forceinline__ void wave_rowdots(const typename Tr<T>::c* rows, int ld, int first, int last,
                                             int step, const typename Tr<T>::pack* vec, int npk,
                                             typename Tr<T>::c* out, int lane) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  if (npk <= 32) {
    wave_rowdots_short<T, kNt>(rows, ld, first, last, step, vec, npk, out, lane);
    return;
  }
  int b = first;
  for (; b + 3 * step < last; b += 4 * step) {
    const P* r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = reinterpret_cast<const P*>(rows + (int64_t)(b + i * step) * ld);
    C a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = czero<C>();
    int p = lane;
    for (; p + 64 < npk; p += 128) {
      P u[4], w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        u[i] = ldnt<kNt>(r[i] + p);
        w[i] = ldnt<kNt>(r[i] + p + 64);
      }
      const P v0 = vec[p], v1 = vec[p + 64];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pdot(a[i], u[i], v0);
        pdot(a[i], w[i], v1);
      }
    }
    if (p < npk) {
      P u[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) u[i] = ldnt<kNt>(r[i] + p);
      const P v0 = vec[p];
#pragma unroll
      for (int i = 0; i < 4; ++i) pdot(a[i], u[i], v0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = wave_sum(a[i]);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) out[b + i * step] = a[i];
    }
  }
  for (; b < last; b += step) {
    const P* r0 = reinterpret_cast<const P*>(rows + (int64_t)b * ld);
    C a0 = czero<C>(), a1 = czero<C>();
    int p = lane;
    for (; p + 64 < npk; p += 128) {
      const P u0 = ldnt<kNt>(r0 + p), u1 = ldnt<kNt>(r0 + p + 64);
      pdot(a0, u0, vec[p]);
      pdot(a1, u1, vec[p + 64]);
    }
    if (p < npk) pdot(a0, ldnt<kNt>(r0 + p), vec[p]);
    a0.x += a1.x;
    a0.y += a1.y;
    a0 = wave_sum(a0);
    if (lane == 0) out[b] = a0;
  }
}

__device__ __forceinline__ float4 shfl_xor_pack(float4 v, int o) {
  return make_float4(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64), __shfl_xor(v.z, o, 64), __shfl_xor(v.w, o, 64));
}
__device__ __forceinline__ double2 shfl_xor_pack(double2 v, int o) {
  return make_double2(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64));
}

// One wavefront, at most 32 column packs: the lanes split into 64 / S groups of S
// (S the smallest power of two >= npk); group g walks rows g, g + 64/S, ..., four in
// flight, and the groups' partial sums meet in a butterfly.  acc[0] of lane p < npk
// receives pack p (acc[1] is zero).
template <typename T>
__device__ __forceinline__ void wave_colaxpy_grouped(const typename Tr<T>::c* rows, int ld, int nrows,
                                                     const typename Tr<T>::c* coef, int npk, int lane,
                                                     typename Tr<T>::pack (&acc)[kColPacks]) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  int S = 1;
  while (S < npk) S <<= 1;
  const int G = 64 / S;
  const int g = lane / S, c = lane - g * S;
  const bool in = c < npk;
  P a = pzero<P>();
  for (int b0 = g; b0 < nrows; b0 += 4 * G) {
    P u[4];
    C cf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = b0 + G * i;
      const bool ok = b < nrows;
      u[i] = (in && ok) ? reinterpret_cast<const P*>(rows + (int64_t)b * ld)[c] : pzero<P>();
      cf[i] = ok ? coef[b] : czero<C>();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) paxpy(a, u[i], cf[i]);
  }
  for (int o = S; o < 64; o <<= 1) a = padd(a, shfl_xor_pack(a, o));
  acc[0] = a;
#pragma unroll
  for (int j = 1; j < kColPacks; ++j) acc[j] = pzero<P>();
}

// acc[j] (column packs base + tid + NT j) += sum_b rows[b][.] * coef[b];
// four rows per iteration.  A single wavefront with at most 32 packs takes the
// grouped form above (acc must then start at zero).
template <typename T, int NT>
__device__ __forceinline__ void block_colaxpy(const typename Tr<T>::c* rows, int ld, int nrows,
                                              const typename Tr<T>::c* coef, int npk, int base, int tid,
                                              typename Tr<T>::pack (&acc)[kColPacks]) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  constexpr bool kNt = NT >= 256;
  if constexpr (NT == 64) {
    if (base == 0 && npk <= 32) {
      wave_colaxpy_grouped<T>(rows, ld, nrows, coef, npk, tid, acc);
      return;
    }
  }
  const int p0 = base + tid;
  bool in[kColPacks];
#pragma unroll
  for (int j = 0; j < kColPacks; ++j) in[j] = p0 + NT * j < npk;
  int b = 0;
  for (; b + 3 < nrows; b += 4) {
    P u[4][kColPacks];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const P* r = reinterpret_cast<const P*>(rows + (int64_t)(b + i) * ld);
#pragma unroll
      for (int j = 0; j < kColPacks; ++j) u[i][j] = in[j] ? ldnt<kNt>(r + p0 + NT * j) : pzero<P>();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const C c = coef[b + i];
#pragma unroll
      for (int j = 0; j < kColPacks; ++j) paxpy(acc[j], u[i][j], c);
    }
  }
  for (; b < nrows; ++b) {
    const P* r = reinterpret_cast<const P*>(rows + (int64_t)b * ld);
    const C c = coef[b];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j)
      if (in[j]) paxpy(acc[j], ldnt<kNt>(r + p0 + NT * j), c);
  }
}

// out(m, n) = sum_k a(m, k) * b(k, n) for m < M, n < N: a small complex product
// computed by the whole workgroup in tiles of four rows per thread, n across
// threads, so that a(m, k) is a broadcast load shared by the four accumulators and
// b(k, n) a coalesced load.
template <typename C, int NT, class FA, class FB, class FO>
__device__ __forceinline__ void tile_product(int M, int N, int K, FA a, FB b, FO out, int tid) {
  const int tasks = (M + 3) / 4 * N;
  for (int task = tid; task < tasks; task += NT) {
    const int m0 = task / N * 4, n = task - task / N * N;
    C acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = czero<C>();
    if (m0 + 3 < M) {
      // KU values of K per step, all operands loaded before the multiply-adds: with
      // operands in global memory each step costs about one memory latency
      constexpr int KU = NT <= 128 ? kSmallKUnroll : 2;
      int k = 0;
      for (; k + KU - 1 < K; k += KU) {
        C bv[KU], av[4][KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) bv[j] = b(k + j, n);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int j = 0; j < KU; ++j) av[u][j] = a(m0 + u, k + j);
#pragma unroll
        for (int j = 0; j < KU; ++j)
#pragma unroll
          for (int u = 0; u < 4; ++u) cfma(acc[u], av[u][j], bv[j]);
      }
      for (; k < K; ++k) {
        const C b0 = b(k, n);
#pragma unroll
        for (int u = 0; u < 4; ++u) cfma(acc[u], a(m0 + u, k), b0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) out(m0 + u, n, acc[u]);
    } else {
      for (int k = 0; k < K; ++k) {
        const C b0 = b(k, n);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (m0 + u < M) cfma(acc[u], a(m0 + u, k), b0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (m0 + u < M) out(m0 + u, n, acc[u]);
    }
  }
}

__device__ __forceinline__ void atomic_add_c(float2* p, float2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}
__device__ __forceinline__ void atomic_add_c(double2* p, double2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}

// ------------------------------------------------------------------ aggregation

// Streaming phase over rows [b0, b1) of U^beta^T and the core: y = U^beta^T x
// (row-dots), then t = core^T y (column axpy) written as packs to `t_out` -- LDS for
// a whole item, the unit's partial-sum block in global memory for a row block of a
// split item.  t[q], q = theta' r_phi + phi'.
template <typename T, int NT>
__device__ __forceinline__ void agg_stream(const typename Tr<T>::c* __restrict__ fac, const TuckItem& it,
                                           const Lds<T>& L, unsigned char* smem, int nrhs, int r,
                                           const typename Tr<T>::c* __restrict__ x, int b0, int b1,
                                           typename Tr<T>::c* t_out) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  constexpr int E = Tr<T>::E;
  C* xs = reinterpret_cast<C*>(smem);
  C* ys = xs + L.r1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = it.nb, Q = it.rt * it.rp;
  const int nbp = round_up(nb, E);

  // x of the group into LDS (zero padded to whole packs)
  for (int n = tid; n < nbp; n += NT) xs[n] = n < nb ? x[(it.row0 + n) * nrhs + r] : czero<C>();
  __syncthreads();

  // y = U^beta^T x (rows b0 .. b1 - 1)
  wave_rowdots<T, (NT >= 256)>(fac + it.off_ubt, it.ld_ub, b0 + wave, b1, (NT / 64), reinterpret_cast<const P*>(xs), nbp / E,
                  ys, lane);
  __syncthreads();

  // t = core^T y over the same rows; t_out may alias x, which is no longer read
  const int qpk = round_up(Q, E) / E;
  for (int base = 0; base < qpk; base += NT * kColPacks) {
    P acc[kColPacks];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) acc[j] = pzero<P>();
    block_colaxpy<T, NT>(fac + it.off_core + (int64_t)b0 * it.ld_c, it.ld_c, b1 - b0, ys + b0, qpk, base, tid,
                         acc);
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) {
      const int p = base + tid + NT * j;
      if (p < qpk) reinterpret_cast<P*>(t_out)[p] = acc[j];
    }
  }
}

// The two angular products of the aggregation, F = U^theta t U^phi^T, with the
// factors at `ut` [n_theta][r_theta] and `upt` [r_phi][n_phi] (global memory or LDS).
template <typename C, int NT>
__device__ __forceinline__ void agg_angular_products(const TuckItem& it, int n_theta, int n_phi, int nrhs,
                                                     const C* ts, C* t3, const C* ut, const C* upt, C* Fo,
                                                     int tid) {
  const int rt = it.rt, rp = it.rp;
  if (it.theta_first) {
    // t3[i][c] = sum_a U^theta[i][a] t[a][c]           (n_theta x r_phi)
    tile_product<C, NT>(
        n_theta, rp, rt, [&](int i, int a) { return ut[i * rt + a]; }, [&](int a, int c) { return ts[a * rp + c]; },
        [&](int i, int c, C v) { t3[i * rp + c] = v; }, tid);
    __syncthreads();
    // F[i][j] = sum_c t3[i][c] U^phi[j][c]
    tile_product<C, NT>(
        n_theta, n_phi, rp, [&](int i, int c) { return t3[i * rp + c]; },
        [&](int c, int j) { return upt[c * n_phi + j]; },
        [&](int i, int j, C v) { Fo[(int64_t)(i * n_phi + j) * nrhs] = v; }, tid);
  } else {
    // t3[a][j] = sum_c t[a][c] U^phi[j][c]             (r_theta x n_phi)
    tile_product<C, NT>(
        rt, n_phi, rp, [&](int a, int c) { return ts[a * rp + c]; }, [&](int c, int j) { return upt[c * n_phi + j]; },
        [&](int a, int j, C v) { t3[a * n_phi + j] = v; }, tid);
    __syncthreads();
    // F[i][j] = sum_a U^theta[i][a] t3[a][j]
    tile_product<C, NT>(
        n_theta, n_phi, rt, [&](int i, int a) { return ut[i * rt + a]; },
        [&](int a, int j) { return t3[a * n_phi + j]; },
        [&](int i, int j, C v) { Fo[(int64_t)(i * n_phi + j) * nrhs] = v; }, tid);
  }
}

// Angular phase: F = U^theta t U^phi^T from t in LDS (`ts`); the intermediate uses
// LDS region r2.
template <typename T, int NT>
__device__ __forceinline__ void agg_angular(const typename Tr<T>::c* __restrict__ fac, const TuckItem& it,
                                            const Lds<T>& L, unsigned char* smem, const typename Tr<T>::c* ts,
                                            int n_theta, int n_phi, int nrhs, int r,
                                            typename Tr<T>::c* __restrict__ F) {
  using C = typename Tr<T>::c;
  C* t3 = reinterpret_cast<C*>(smem) + L.r1;
  const int tid = threadIdx.x;
  const int rt = it.rt, rp = it.rp;
  const C* ut = fac + it.off_ut;    // [n_theta][rt]
  const C* upt = fac + it.off_upt;  // [rp][n_phi]
  const int ndir = n_theta * n_phi;
  C* Fo = F + ((int64_t)it.frow * ndir) * nrhs + r;
  if (it.ident) {  // truncated-SVD item: t already holds the directions
    for (int i = tid; i < ndir; i += NT) Fo[(int64_t)i * nrhs] = ts[i];
    return;
  }
  if (L.sa) {
    // the factors into LDS (one load latency for both) after the r1 and r2 regions:
    // the products then take one LDS access per K step instead of a memory latency
    C* s_ut = reinterpret_cast<C*>(smem) + L.r1 + L.r2;
    C* s_upt = s_ut + round_up(n_theta * rt, 2);
    for (int q = tid; q < n_theta * rt; q += NT) s_ut[q] = ut[q];
    for (int q = tid; q < rp * n_phi; q += NT) s_upt[q] = upt[q];
    __syncthreads();
    agg_angular_products<C, NT>(it, n_theta, n_phi, nrhs, ts, t3, s_ut, s_upt, Fo, tid);
  } else {
    agg_angular_products<C, NT>(it, n_theta, n_phi, nrhs, ts, t3, ut, upt, Fo, tid);
  }
}

// --------------------------------------------------------------- disaggregation

// Angular phase: S = U^theta^T conj(G) U^phi, written with its pack padding to
// `S2` in LDS.  With zero_v the item also clears its rows of V.
template <typename T, int NT>
__device__ __forceinline__ void dis_angular(const typename Tr<T>::c* __restrict__ fac, const TuckItem& it,
                                            const Lds<T>& L, unsigned char* smem, int n_theta, int n_phi,
                                            int nrhs, int r, const typename Tr<T>::c* __restrict__ Gin,
                                            typename Tr<T>::c* S2, bool zero_v, typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  constexpr int E = Tr<T>::E;
  C* s1 = reinterpret_cast<C*>(smem);
  const int tid = threadIdx.x;
  const int ndir = n_theta * n_phi;
  const int rt = it.rt, rp = it.rp, Q = rt * rp;
  const C* ut = fac + it.off_ut;  // [n_theta][rt]
  const C* up = fac + it.off_up;  // [n_phi][rp]
  const C* Gi = Gin + ((int64_t)it.frow * ndir) * nrhs + r;
  if (zero_v)
    for (int n = tid; n < it.nb; n += NT) V[(it.row0 + n) * nrhs + r] = czero<C>();
  // the angular order mirrors the aggregation choice
  if (it.ident) {  // truncated-SVD item: S2 is conj(G) itself
    for (int q = tid; q < Q; q += NT) S2[q] = conjc(Gi[(int64_t)q * nrhs]);
  } else if (L.sd) {
    // conj(G) and the first product's factor into LDS after the s regions (one load
    // latency), then the second product's factor in their place
    C* gs = reinterpret_cast<C*>(smem) + L.s1 + L.s2 + L.s3;
    C* fs = gs + round_up(ndir, 2);
    for (int q = tid; q < ndir; q += NT) gs[q] = conjc(Gi[(int64_t)q * nrhs]);
    if (!it.theta_first) {
      for (int q = tid; q < n_theta * rt; q += NT) fs[q] = ut[q];
      __syncthreads();
      tile_product<C, NT>(
          rt, n_phi, n_theta, [&](int a, int i) { return fs[i * rt + a]; },
          [&](int i, int j) { return gs[i * n_phi + j]; }, [&](int a, int j, C v) { s1[a * n_phi + j] = v; }, tid);
      __syncthreads();
      for (int q = tid; q < n_phi * rp; q += NT) gs[q] = up[q];
      __syncthreads();
      tile_product<C, NT>(
          rt, rp, n_phi, [&](int a, int j) { return s1[a * n_phi + j]; }, [&](int j, int c) { return gs[j * rp + c]; },
          [&](int a, int c, C v) { S2[a * rp + c] = v; }, tid);
    } else {
      for (int q = tid; q < n_phi * rp; q += NT) fs[q] = up[q];
      __syncthreads();
      tile_product<C, NT>(
          n_theta, rp, n_phi, [&](int i, int j) { return gs[i * n_phi + j]; },
          [&](int j, int c) { return fs[j * rp + c]; }, [&](int i, int c, C v) { s1[i * rp + c] = v; }, tid);
      __syncthreads();
      for (int q = tid; q < n_theta * rt; q += NT) gs[q] = ut[q];
      __syncthreads();
      tile_product<C, NT>(
          rt, rp, n_theta, [&](int a, int i) { return gs[i * rt + a]; }, [&](int i, int c) { return s1[i * rp + c]; },
          [&](int a, int c, C v) { S2[a * rp + c] = v; }, tid);
    }
  } else if (!it.theta_first) {
    // s1[a][j] = sum_i U^theta[i][a] conj(G[i][j])     (r_theta x n_phi)
    tile_product<C, NT>(
        rt, n_phi, n_theta, [&](int a, int i) { return ut[i * rt + a]; },
        [&](int i, int j) { return conjc(Gi[(int64_t)(i * n_phi + j) * nrhs]); },
        [&](int a, int j, C v) { s1[a * n_phi + j] = v; }, tid);
    __syncthreads();
    // S[a][c] = sum_j s1[a][j] U^phi[j][c]
    tile_product<C, NT>(
        rt, rp, n_phi, [&](int a, int j) { return s1[a * n_phi + j]; }, [&](int j, int c) { return up[j * rp + c]; },
        [&](int a, int c, C v) { S2[a * rp + c] = v; }, tid);
  } else {
    // s1[i][c] = sum_j conj(G[i][j]) U^phi[j][c]       (n_theta x r_phi)
    tile_product<C, NT>(
        n_theta, rp, n_phi, [&](int i, int j) { return conjc(Gi[(int64_t)(i * n_phi + j) * nrhs]); },
        [&](int j, int c) { return up[j * rp + c]; }, [&](int i, int c, C v) { s1[i * rp + c] = v; }, tid);
    __syncthreads();
    // S[a][c] = sum_i U^theta[i][a] s1[i][c]
    tile_product<C, NT>(
        rt, rp, n_theta, [&](int a, int i) { return ut[i * rt + a]; }, [&](int i, int c) { return s1[i * rp + c]; },
        [&](int a, int c, C v) { S2[a * rp + c] = v; }, tid);
  }
  for (int o = Q + tid; o < round_up(Q, E); o += NT) S2[o] = czero<C>();  // pack padding
}

// Streaming phase over rows [b0, b1): s = core S (row-dots) with S in LDS region s2,
// then v[n] = sum_b U^beta[n][b] s[b] (column axpy).  A whole item adds conj(v) to V
// (atomic adds); a row block of a split item (part_out != nullptr) stores v as its
// partial-sum block.
template <typename T, int NT>
__device__ __forceinline__ void dis_stream(const typename Tr<T>::c* __restrict__ fac, const TuckItem& it,
                                           const Lds<T>& L, unsigned char* smem, int nrhs, int r, int b0, int b1,
                                           typename Tr<T>::c* part_out, typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  constexpr int E = Tr<T>::E;
  C* S2 = reinterpret_cast<C*>(smem) + L.s1;
  C* s3 = S2 + L.s2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Q = it.rt * it.rp;
  // s[b] = sum_q core[b][q] S[q]
  wave_rowdots<T, (NT >= 256)>(fac + it.off_core, it.ld_c, b0 + wave, b1, (NT / 64), reinterpret_cast<const P*>(S2),
                  round_up(Q, E) / E, s3, lane);
  __syncthreads();
  // V[n] += conj(sum_b U^beta[n][b] s[b])
  const int nb = it.nb;
  const int npk = round_up(nb, E) / E;
  C* Vo = V + it.row0 * nrhs + r;
  for (int base = 0; base < npk; base += NT * kColPacks) {
    P acc[kColPacks];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) acc[j] = pzero<P>();
    block_colaxpy<T, NT>(fac + it.off_ubt + (int64_t)b0 * it.ld_ub, it.ld_ub, b1 - b0, s3 + b0, npk, base, tid,
                         acc);
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) {
      const int p = base + tid + NT * j;
      if (p < npk && part_out) {
        reinterpret_cast<P*>(part_out)[p] = acc[j];
      } else if (p < npk) {
        const C* vals = reinterpret_cast<const C*>(&acc[j]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int n = p * E + e;
          if (n < nb) atomic_add_c(Vo + (int64_t)n * nrhs, conjc(vals[e]));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------- kernels

// Aggregation of one work unit: a whole item (stream, angular phase, F written) or a
// row block of a split item (its partial t stored for the finishing kernel).
template <typename T, int NT>
__device__ __forceinline__ void agg_unit(const typename Tr<T>::c* __restrict__ fac, const TuckItem* items,
                                         const TuckUnit& u, const TuckSplit* splits, const Lds<T>& L,
                                         unsigned char* smem, int n_theta, int n_phi, int nrhs, int r,
                                         const typename Tr<T>::c* __restrict__ x, typename Tr<T>::c* __restrict__ F,
                                         typename Tr<T>::c* part, int64_t part_stride) {
  using C = typename Tr<T>::c;
  const TuckItem it = items[u.item];
  if (u.split < 0) {
    C* ts = reinterpret_cast<C*>(smem);  // t over x
    agg_stream<T, NT>(fac, it, L, smem, nrhs, r, x, 0, it.rb, ts);
    __syncthreads();
    agg_angular<T, NT>(fac, it, L, smem, ts, n_theta, n_phi, nrhs, r, F);
  } else {
    const TuckSplit sp = splits[u.split];
    agg_stream<T, NT>(fac, it, L, smem, nrhs, r, x, u.b0, u.b1,
                      part + r * part_stride + sp.agg_off + (int64_t)u.sub * sp.q_pad);
  }
}

// Disaggregation of one work unit: angular phase, then the stream over the unit's
// rows; a whole item adds into V, a row block stores its partial v.
template <typename T, int NT>
__device__ __forceinline__ void dis_unit(const typename Tr<T>::c* __restrict__ fac, const TuckItem* items,
                                         const TuckUnit& u, const TuckSplit* splits, const Lds<T>& L,
                                         unsigned char* smem, int n_theta, int n_phi, int nrhs, int r,
                                         const typename Tr<T>::c* __restrict__ G, typename Tr<T>::c* __restrict__ V,
                                         typename Tr<T>::c* part, int64_t part_stride) {
  using C = typename Tr<T>::c;
  const TuckItem it = items[u.item];
  C* dst = nullptr;
  if (u.split >= 0) {
    const TuckSplit sp = splits[u.split];
    dst = part + r * part_stride + sp.dis_off + (int64_t)u.sub * sp.nb_pad;
  }
  dis_angular<T, NT>(fac, it, L, smem, n_theta, n_phi, nrhs, r, G, reinterpret_cast<C*>(smem) + L.s1, false, V);
  __syncthreads();
  dis_stream<T, NT>(fac, it, L, smem, nrhs, r, u.b0, u.b1, dst, V);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void tucker_agg_kernel(const typename Tr<T>::c* __restrict__ fac,
                                                        const TuckItem* __restrict__ items,
                                                        const TuckUnit* __restrict__ units,
                                                        const TuckSplit* __restrict__ splits,
                                                        const int32_t* __restrict__ order, TuckMax mx, int n_theta,
                                                        int n_phi, int nrhs,
                                                        const typename Tr<T>::c* __restrict__ x,
                                                        typename Tr<T>::c* __restrict__ F, typename Tr<T>::c* part,
                                                        int64_t part_stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  const TuckUnit u = units[order[blockIdx.x]];
  agg_unit<T, NT>(fac, items, u, splits, Lds<T>(mx), smem, n_theta, n_phi, nrhs, blockIdx.y, x, F,
                  part, part_stride);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void tucker_dis_kernel(const typename Tr<T>::c* __restrict__ fac,
                                                        const TuckItem* __restrict__ items,
                                                        const TuckUnit* __restrict__ units,
                                                        const TuckSplit* __restrict__ splits,
                                                        const int32_t* __restrict__ order, TuckMax mx, int n_theta,
                                                        int n_phi, int nrhs,
                                                        const typename Tr<T>::c* __restrict__ G,
                                                        typename Tr<T>::c* __restrict__ V, typename Tr<T>::c* part,
                                                        int64_t part_stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  const TuckUnit u = units[order[blockIdx.x]];
  dis_unit<T, NT>(fac, items, u, splits, Lds<T>(mx), smem, n_theta, n_phi, nrhs, blockIdx.y, G, V,
                  part, part_stride);
}

// One launch for a whole aggregation + disaggregation pass: work-list entry e is
// the aggregation of unit e if e >= 0 and the disaggregation of unit ~e otherwise.
// Both stages' units interleave in one longest-first list, so small units of either
// stage fill the end of the launch.  The launch is persistent: as many workgroups as
// the CUs hold at once, each taking the next entry (of n_list per right-hand side) from
// the work counter `next`, which the V-zeroing kernel before it sets to zero.  On
// layouts of many small units this keeps every CU full; with one workgroup per entry
// the hardware refilled a CU's free slot only tens of microseconds after a unit ended.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void tucker_pass_kernel(const typename Tr<T>::c* __restrict__ fac,
                                                         const TuckItem* __restrict__ items,
                                                         const TuckUnit* __restrict__ units,
                                                         const TuckSplit* __restrict__ splits,
                                                         const int32_t* __restrict__ list, int n_list, TuckMax mx,
                                                         int n_theta, int n_phi, int nrhs,
                                                         const typename Tr<T>::c* __restrict__ x,
                                                         typename Tr<T>::c* __restrict__ F,
                                                         const typename Tr<T>::c* __restrict__ G,
                                                         typename Tr<T>::c* __restrict__ V, typename Tr<T>::c* part,
                                                         int64_t part_stride, int32_t* __restrict__ next) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t take;
  const Lds<T> L(mx);
  const int total = n_list * nrhs;
  for (;;) {
    if (threadIdx.x == 0) take = atomicAdd(next, 1);
    __syncthreads();
    const int i = take;
    if (i >= total) break;  // uniform: every wavefront leaves
    const int r = i / n_list;
    const int32_t e = list[i - r * n_list];
    if (e >= 0)
      agg_unit<T, NT>(fac, items, units[e], splits, L, smem, n_theta, n_phi, nrhs, r, x, F, part, part_stride);
    else
      dis_unit<T, NT>(fac, items, units[~e], splits, L, smem, n_theta, n_phi, nrhs, r, G, V, part, part_stride);
    __syncthreads();  // the unit's last LDS reads and `take` are done before the next entry
  }
}

// Finishing kernel of the split items, after the units: blocks [0, n_agg) sum the
// partial t of split entry blockIdx.x (in block order, so the result does not depend
// on the schedule) and run the angular phase into F; blocks [n_agg, gridDim.x) sum
// the partial v of split entry blockIdx.x - n_agg and add conj(v) to V.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void tucker_finish_kernel(const typename Tr<T>::c* __restrict__ fac,
                                                           const TuckItem* __restrict__ items,
                                                           const TuckSplit* __restrict__ splits, int n_agg,
                                                           TuckMax mx, int n_theta, int n_phi, int nrhs,
                                                           const typename Tr<T>::c* __restrict__ part,
                                                           int64_t part_stride, typename Tr<T>::c* __restrict__ F,
                                                           typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  constexpr int E = Tr<T>::E;
  extern __shared__ __align__(16) unsigned char smem[];
  const int r = blockIdx.y, tid = threadIdx.x;
  const bool agg = (int)blockIdx.x < n_agg;
  const TuckSplit sp = splits[agg ? blockIdx.x : blockIdx.x - n_agg];
  const TuckItem it = items[sp.item];
  const C* base = part + r * part_stride;
  if (agg) {
    const int Q = it.rt * it.rp;
    C* ts = reinterpret_cast<C*>(smem);
    for (int q = tid; q < round_up(Q, E); q += NT) {
      C acc = czero<C>();
      if (q < Q)
        for (int s = 0; s < sp.n_parts; ++s) {
          const C v = base[sp.agg_off + (int64_t)s * sp.q_pad + q];
          acc.x += v.x;
          acc.y += v.y;
        }
      ts[q] = acc;
    }
    __syncthreads();
    agg_angular<T, NT>(fac, it, Lds<T>(mx), smem, ts, n_theta, n_phi, nrhs, r, F);
  } else {
    C* Vo = V + it.row0 * nrhs + r;
    for (int n = tid; n < it.nb; n += NT) {
      C acc = czero<C>();
      for (int s = 0; s < sp.n_parts; ++s) {
        const C v = base[sp.dis_off + (int64_t)s * sp.nb_pad + n];
        acc.x += v.x;
        acc.y += v.y;
      }
      atomic_add_c(Vo + (int64_t)n * nrhs, conjc(acc));
    }
  }
}

// v[0 .. n) = 0; with `counter`, also the pass kernel's work counter.
template <typename C>
__global__ __launch_bounds__(256) void zero_kernel(C* __restrict__ v, int64_t n, int32_t* __restrict__ counter) {
  if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v[i] = czero<C>();
}

template <typename C>
hipError_t zero(C* v, int64_t n, hipStream_t s, int32_t* counter = nullptr) {
  if (n <= 0 && !counter) return hipSuccess;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(zero_kernel<C>, dim3((unsigned)blocks), dim3(256), 0, s, v, n, counter);
  return hipGetLastError();
}

// Grid of a persistent launch: the workgroups of `kernel` the CUs hold at once (by
// its registers and LDS), at most one per work entry.
template <typename K>
hipError_t persistent_grid(K kernel, int threads, size_t lds, int64_t entries, unsigned* blocks) {
  int dev = 0, n_cu = 0, per_cu = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), threads,
                                                        lds)) != hipSuccess)
    return e;
  *blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(entries, (int64_t)std::max(per_cu, 1) * n_cu));
  return hipSuccess;
}

// One row per blockIdx.x, the row's elements split over blockIdx.y.
template <typename C>
__global__ __launch_bounds__(256) void zero_rows_kernel(C* __restrict__ base, const int32_t* __restrict__ rows,
                                                        int64_t row_elems) {
  C* row = base + (int64_t)rows[blockIdx.x] * row_elems;
  for (int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x; i < row_elems; i += (int64_t)gridDim.y * 256)
    row[i] = czero<C>();
}

}  // namespace

hipError_t launch_zero_rows(size_t elem_bytes, void* base, const int32_t* rows, int n_rows, int64_t row_elems,
                            hipStream_t s) {
  if (n_rows <= 0 || row_elems <= 0) return hipSuccess;
  const unsigned ny = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (row_elems + 2047) / 2048), 1024);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(zero_rows_kernel<Tr<double>::c>, dim3((unsigned)n_rows, ny), dim3(256), 0, s,
                       static_cast<Tr<double>::c*>(base), rows, row_elems);
  else if (elem_bytes == 8)
    hipLaunchKernelGGL(zero_rows_kernel<Tr<float>::c>, dim3((unsigned)n_rows, ny), dim3(256), 0, s,
                       static_cast<Tr<float>::c*>(base), rows, row_elems);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
size_t tucker_lds_bytes(const TuckMax& mx) {
  return Lds<T>(mx).bytes();
}

// Workgroup sizes a launch may take.
#define TFMM_NT_SWITCH(threads, ...) \
  switch (threads) {                  \
    case 64: {                        \
      constexpr int NT = 64;          \
      __VA_ARGS__;                    \
      break;                          \
    }                                 \
    case 128: {                       \
      constexpr int NT = 128;         \
      __VA_ARGS__;                    \
      break;                          \
    }                                 \
    case 256: {                       \
      constexpr int NT = 256;         \
      __VA_ARGS__;                    \
      break;                          \
    }                                 \
    case 512: {                       \
      constexpr int NT = 512;         \
      __VA_ARGS__;                    \
      break;                          \
    }                                 \
    default:                          \
      return hipErrorInvalidValue;    \
  }

template <typename T>
hipError_t launch_finish(const TuckPlan& pl, int threads, int n_agg, int n_dis, int n_theta, int n_phi, int nrhs,
                         void* F, void* V, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_agg + n_dis == 0) return hipSuccess;
  const size_t lds = n_agg ? Lds<T>(pl.mx).agg_bytes() : 0;
  // n_dis > 0 with n_agg == 0 runs the disaggregation blocks only: splits from 0
  const TuckSplit* sp = pl.splits;
  TFMM_NT_SWITCH(threads,
                 hipLaunchKernelGGL((tucker_finish_kernel<T, NT>), dim3(n_agg + n_dis, nrhs), dim3(NT), lds, s,
                                    static_cast<const C*>(pl.factors), pl.items, sp, n_agg, pl.mx, n_theta, n_phi,
                                    nrhs, static_cast<const C*>(pl.part), pl.part_stride, static_cast<C*>(F),
                                    static_cast<C*>(V)))
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tucker_agg(const TuckPlan& pl, int threads, int n_theta, int n_phi, int nrhs, const void* x,
                             void* F, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (pl.n_units == 0) return hipSuccess;
  if (pl.n_splits > 0 && pl.part == nullptr) return hipErrorInvalidValue;
  TFMM_NT_SWITCH(threads,
                 hipLaunchKernelGGL((tucker_agg_kernel<T, NT>), dim3(pl.n_units, nrhs), dim3(NT),
                                    Lds<T>(pl.mx).agg_bytes(), s, static_cast<const C*>(pl.factors), pl.items,
                                    pl.units, pl.splits, pl.order, pl.mx, n_theta, n_phi, nrhs,
                                    static_cast<const C*>(x), static_cast<C*>(F), static_cast<C*>(pl.part),
                                    pl.part_stride))
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish<T>(pl, threads, pl.n_splits, 0, n_theta, n_phi, nrhs, F, nullptr, s);
}

template <typename T>
hipError_t launch_tucker_disagg(const TuckPlan& pl, int threads, int n_theta, int n_phi, int nrhs, const void* G,
                                void* V, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512) return hipErrorInvalidValue;
  if (pl.n_splits > 0 && pl.part == nullptr) return hipErrorInvalidValue;
  hipError_t e = zero(static_cast<C*>(V), pl.n_basis * nrhs, s);
  if (e != hipSuccess || pl.n_units == 0) return e;
  TFMM_NT_SWITCH(threads,
                 hipLaunchKernelGGL((tucker_dis_kernel<T, NT>), dim3(pl.n_units, nrhs), dim3(NT),
                                    Lds<T>(pl.mx).dis_bytes(), s, static_cast<const C*>(pl.factors), pl.items,
                                    pl.units, pl.splits, pl.order, pl.mx, n_theta, n_phi, nrhs,
                                    static_cast<const C*>(G), static_cast<C*>(V), static_cast<C*>(pl.part),
                                    pl.part_stride))
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish<T>(pl, threads, 0, pl.n_splits, n_theta, n_phi, nrhs, nullptr, V, s);
}

template <typename T>
hipError_t launch_tucker_pass(const TuckPlan& pl, int threads, int n_theta, int n_phi, int nrhs, const void* x,
                              void* F, const void* G, void* V, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512) return hipErrorInvalidValue;
  if (pl.n_splits > 0 && pl.part == nullptr) return hipErrorInvalidValue;
  if (pl.next == nullptr) return hipErrorInvalidValue;
  hipError_t e = zero(static_cast<C*>(V), pl.n_basis * nrhs, s, pl.next);
  if (e != hipSuccess || pl.n_units == 0) return e;
  const int n_list = 2 * pl.n_units;
  const size_t lds = Lds<T>(pl.mx).bytes();
  unsigned blocks = 0;
  TFMM_NT_SWITCH(threads, e = persistent_grid(&tucker_pass_kernel<T, NT>, NT, lds, (int64_t)n_list * nrhs, &blocks))
  if (e != hipSuccess) return e;
  TFMM_NT_SWITCH(threads,
                 hipLaunchKernelGGL((tucker_pass_kernel<T, NT>), dim3(blocks), dim3(NT), lds, s,
                                    static_cast<const C*>(pl.factors), pl.items, pl.units, pl.splits, pl.pass_list,
                                    n_list, pl.mx, n_theta, n_phi, nrhs, static_cast<const C*>(x),
                                    static_cast<C*>(F), static_cast<const C*>(G), static_cast<C*>(V),
                                    static_cast<C*>(pl.part), pl.part_stride, pl.next))
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish<T>(pl, threads, pl.n_splits, pl.n_splits, n_theta, n_phi, nrhs, F, V, s);
}

template size_t tucker_lds_bytes<float>(const TuckMax&);
template size_t tucker_lds_bytes<double>(const TuckMax&);
template hipError_t launch_tucker_agg<float>(const TuckPlan&, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_tucker_agg<double>(const TuckPlan&, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_tucker_disagg<float>(const TuckPlan&, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_tucker_disagg<double>(const TuckPlan&, int, int, int, int, const void*, void*,
                                                 hipStream_t);
template hipError_t launch_tucker_pass<float>(const TuckPlan&, int, int, int, int, const void*, void*, const void*,
                                              void*, hipStream_t);
template hipError_t launch_tucker_pass<double>(const TuckPlan&, int, int, int, int, const void*, void*, const void*,
                                               void*, hipStream_t);

}  // namespace tuckfmm
