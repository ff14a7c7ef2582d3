// Tucker-format aggregation and disaggregation (Section II.C, Figs. 2(b) and 3(b)).
//
// One 256-thread workgroup (four 64-wide wavefronts) per work item; the work list
// is sorted by decreasing cost, so the hardware dispatcher hands out the largest
// items first (longest-processing-time order).  The two large operands of every
// item -- U^beta and the core -- are streamed once from HBM with 16-byte coalesced
// loads; everything else stays in LDS.
//
// Aggregation of item (g, alpha), contraction order chosen per item on the host:
//   y[b]    = sum_n U^beta[n][b] x[n]          row-dot of each U^beta^T row
//                                              (one wavefront per row, lane-strided,
//                                              butterfly reduction)
//   t[q]    = sum_b core[b][q] y[b]            column axpy over the core rows
//                                              (one thread per column pack)
//   F[i,j]  = sum U^theta[i][a] U^phi[j][c] t[a, c]   two small LDS products
// Disaggregation of group g (both polarisations, summed as in eq. (5)):
//   S[a,c]  = sum U^theta[i][a] U^phi[j][c] conj(G[i,j])   small LDS products
//   s[b]    = sum_q core[b][q] S[q]            row-dot of each core row
//   V[n]    = conj(sum_alpha sum_b U^beta[n][b] s[b])      column axpy over U^beta^T
#include <hip/hip_runtime.h>
#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kColPacks = 2;  // column packs per thread per chunk in the axpy stages

template <typename T>
struct AggLds {
  int regA, y, t2;  // element counts of each region (complex)
  __host__ __device__ explicit AggLds(const TuckMax& mx) {
    constexpr int E = Tr<T>::E;
    regA = round_up(max(round_up(mx.nb, E), mx.t3), 2);
    y = round_up(mx.rb, 2);
    t2 = round_up(round_up(mx.q, E), 2);
  }
  __host__ __device__ size_t bytes() const { return size_t(regA + y + t2) * sizeof(typename Tr<T>::c); }
};

template <typename T>
struct DisLds {
  int s1, s2, s3;
  __host__ __device__ explicit DisLds(const TuckMax& mx) {
    constexpr int E = Tr<T>::E;
    s1 = round_up(mx.t3, 2);
    s2 = round_up(round_up(mx.q, E), 2);   // per polarisation
    s3 = round_up(mx.rb, 2);               // per polarisation
  }
  __host__ __device__ size_t bytes() const { return size_t(s1 + 2 * s2 + 2 * s3) * sizeof(typename Tr<T>::c); }
};

// out[b] = sum_k rows[b][k] * vec[k] for b = first, first + step, ...  (one wavefront
// per row).  rows are 16-byte aligned with npk packs each; vec is an LDS pack array.
template <typename T>
__device__ __forceinline__ void wave_rowdots(const typename Tr<T>::c* rows, int ld, int first, int last,
                                             int step, const typename Tr<T>::pack* vec, int npk,
                                             typename Tr<T>::c* out, int lane) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  int b = first;
  // two rows at a time to keep more loads in flight
  for (; b + step < last; b += 2 * step) {
    const P* r0 = reinterpret_cast<const P*>(rows + (int64_t)b * ld);
    const P* r1 = reinterpret_cast<const P*>(rows + (int64_t)(b + step) * ld);
    C a0 = czero<C>(), a1 = czero<C>();
    int p = lane;
    for (; p + 64 < npk; p += 128) {
      P u0 = r0[p], u1 = r1[p], u2 = r0[p + 64], u3 = r1[p + 64];
      P v0 = vec[p], v1 = vec[p + 64];
      pdot(a0, u0, v0);
      pdot(a1, u1, v0);
      pdot(a0, u2, v1);
      pdot(a1, u3, v1);
    }
    if (p < npk) {
      P v0 = vec[p];
      pdot(a0, r0[p], v0);
      pdot(a1, r1[p], v0);
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
      out[b] = a0;
      out[b + step] = a1;
    }
  }
  if (b < last) {
    const P* r0 = reinterpret_cast<const P*>(rows + (int64_t)b * ld);
    C a0 = czero<C>();
    for (int p = lane; p < npk; p += 64) pdot(a0, r0[p], vec[p]);
    a0 = wave_sum(a0);
    if (lane == 0) out[b] = a0;
  }
}

// acc[j] (column packs base + tid + 256 j) += sum_b rows[b][.] * coef[b]
template <typename T>
__device__ __forceinline__ void block_colaxpy(const typename Tr<T>::c* rows, int ld, int nrows,
                                              const typename Tr<T>::c* coef, int npk, int base, int tid,
                                              typename Tr<T>::pack (&acc)[kColPacks]) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  const int p0 = base + tid;
  bool in[kColPacks];
#pragma unroll
  for (int j = 0; j < kColPacks; ++j) in[j] = p0 + kThreads * j < npk;
  int b = 0;
  for (; b + 1 < nrows; b += 2) {
    const P* r0 = reinterpret_cast<const P*>(rows + (int64_t)b * ld);
    const P* r1 = reinterpret_cast<const P*>(rows + (int64_t)(b + 1) * ld);
    P u[kColPacks], w[kColPacks];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) {
      u[j] = in[j] ? r0[p0 + kThreads * j] : pzero<P>();
      w[j] = in[j] ? r1[p0 + kThreads * j] : pzero<P>();
    }
    const C c0 = coef[b], c1 = coef[b + 1];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) {
      paxpy(acc[j], u[j], c0);
      paxpy(acc[j], w[j], c1);
    }
  }
  if (b < nrows) {
    const P* r0 = reinterpret_cast<const P*>(rows + (int64_t)b * ld);
    const C c0 = coef[b];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j)
      if (in[j]) paxpy(acc[j], r0[p0 + kThreads * j], c0);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void tucker_agg_kernel(
    const typename Tr<T>::c* __restrict__ fac, const TuckItem* __restrict__ items,
    const int32_t* __restrict__ order, TuckMax mx, int n_theta, int n_phi, int nrhs,
    const typename Tr<T>::c* __restrict__ x, typename Tr<T>::c* __restrict__ F) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  constexpr int E = Tr<T>::E;
  extern __shared__ __align__(16) unsigned char smem[];
  const AggLds<T> L(mx);
  C* xs = reinterpret_cast<C*>(smem);
  C* ys = xs + L.regA;
  C* ts = ys + L.y;

  const TuckItem it = items[order[blockIdx.x]];
  const int r = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = it.nb, rb = it.rb, rt = it.rt, rp = it.rp, Q = rt * rp;
  const int nbp = round_up(nb, E);

  // x of the group into LDS (zero padded to whole packs)
  for (int n = tid; n < nbp; n += kThreads)
    xs[n] = n < nb ? x[(it.row0 + n) * nrhs + r] : czero<C>();
  __syncthreads();

  // y = U^beta^T x
  wave_rowdots<T>(fac + it.off_ubt, it.ld_ub, wave, rb, kWaves, reinterpret_cast<const P*>(xs), nbp / E, ys,
                  lane);
  __syncthreads();

  // t = core^T y   (t[q], q = theta' * r_phi + phi')
  const int qpk = round_up(Q, E) / E;
  for (int base = 0; base < qpk; base += kThreads * kColPacks) {
    P acc[kColPacks];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) acc[j] = pzero<P>();
    block_colaxpy<T>(fac + it.off_core, it.ld_c, rb, ys, qpk, base, tid, acc);
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) {
      const int p = base + tid + kThreads * j;
      if (p < qpk) reinterpret_cast<P*>(ts)[p] = acc[j];
    }
  }
  __syncthreads();

  // angular stages; regA (x) is free now
  const C* ut = fac + it.off_ut;    // [n_theta][rt]
  const C* upt = fac + it.off_upt;  // [rp][n_phi]
  C* t3 = xs;
  const int ndir = n_theta * n_phi;
  C* Fo = F + ((int64_t)(it.group * 2 + it.alpha) * ndir) * nrhs + r;
  if (it.theta_first) {
    // t3[i][c] = sum_a U^theta[i][a] t[a][c]           (n_theta x r_phi)
    for (int o = tid; o < n_theta * rp; o += kThreads) {
      const int i = o / rp, c = o - i * rp;
      C acc = czero<C>();
      for (int a = 0; a < rt; ++a) cfma(acc, ut[i * rt + a], ts[a * rp + c]);
      t3[o] = acc;
    }
    __syncthreads();
    // F[i][j] = sum_c t3[i][c] U^phi[j][c]
    for (int o = tid; o < ndir; o += kThreads) {
      const int i = o / n_phi, j = o - i * n_phi;
      C acc = czero<C>();
      for (int c = 0; c < rp; ++c) cfma(acc, t3[i * rp + c], upt[c * n_phi + j]);
      Fo[(int64_t)o * nrhs] = acc;
    }
  } else {
    // t3[a][j] = sum_c t[a][c] U^phi[j][c]             (r_theta x n_phi)
    for (int o = tid; o < rt * n_phi; o += kThreads) {
      const int a = o / n_phi, j = o - a * n_phi;
      C acc = czero<C>();
      for (int c = 0; c < rp; ++c) cfma(acc, ts[a * rp + c], upt[c * n_phi + j]);
      t3[o] = acc;
    }
    __syncthreads();
    // F[i][j] = sum_a U^theta[i][a] t3[a][j]
    for (int o = tid; o < ndir; o += kThreads) {
      const int i = o / n_phi, j = o - i * n_phi;
      C acc = czero<C>();
      for (int a = 0; a < rt; ++a) cfma(acc, ut[i * rt + a], t3[a * n_phi + j]);
      Fo[(int64_t)o * nrhs] = acc;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void tucker_disagg_kernel(
    const typename Tr<T>::c* __restrict__ fac, const TuckItem* __restrict__ items,
    const int32_t* __restrict__ order, TuckMax mx, int n_theta, int n_phi, int nrhs,
    const typename Tr<T>::c* __restrict__ Gin, typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  using P = typename Tr<T>::pack;
  constexpr int E = Tr<T>::E;
  extern __shared__ __align__(16) unsigned char smem[];
  const DisLds<T> L(mx);
  C* s1 = reinterpret_cast<C*>(smem);
  C* s2 = s1 + L.s1;          // [2][L.s2]
  C* s3 = s2 + 2 * L.s2;      // [2][L.s3]

  const int g = order[blockIdx.x];
  const int r = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const TuckItem it0 = items[2 * g], it1 = items[2 * g + 1];
  const int ndir = n_theta * n_phi;

  for (int alpha = 0; alpha < 2; ++alpha) {
    const TuckItem& it = alpha ? it1 : it0;
    const int rt = it.rt, rp = it.rp, Q = rt * rp;
    const C* ut = fac + it.off_ut;  // [n_theta][rt]
    const C* up = fac + it.off_up;  // [n_phi][rp]
    const C* Gi = Gin + ((int64_t)(g * 2 + alpha) * ndir) * nrhs + r;
    C* S2 = s2 + alpha * L.s2;
    // the angular order of disaggregation mirrors the aggregation choice
    if (!it.theta_first) {
      // s1[a][j] = sum_i U^theta[i][a] conj(G[i][j])     (r_theta x n_phi)
      for (int o = tid; o < rt * n_phi; o += kThreads) {
        const int a = o / n_phi, j = o - a * n_phi;
        C acc = czero<C>();
        for (int i = 0; i < n_theta; ++i) cfma(acc, ut[i * rt + a], conjc(Gi[(int64_t)(i * n_phi + j) * nrhs]));
        s1[o] = acc;
      }
      __syncthreads();
      // S2[a][c] = sum_j s1[a][j] U^phi[j][c]
      for (int o = tid; o < Q; o += kThreads) {
        const int a = o / rp, c = o - a * rp;
        C acc = czero<C>();
        for (int j = 0; j < n_phi; ++j) cfma(acc, s1[a * n_phi + j], up[j * rp + c]);
        S2[o] = acc;
      }
    } else {
      // s1[i][c] = sum_j conj(G[i][j]) U^phi[j][c]       (n_theta x r_phi)
      for (int o = tid; o < n_theta * rp; o += kThreads) {
        const int i = o / rp, c = o - i * rp;
        C acc = czero<C>();
        for (int j = 0; j < n_phi; ++j) cfma(acc, up[j * rp + c], conjc(Gi[(int64_t)(i * n_phi + j) * nrhs]));
        s1[o] = acc;
      }
      __syncthreads();
      // S2[a][c] = sum_i U^theta[i][a] s1[i][c]
      for (int o = tid; o < Q; o += kThreads) {
        const int a = o / rp, c = o - a * rp;
        C acc = czero<C>();
        for (int i = 0; i < n_theta; ++i) cfma(acc, ut[i * rt + a], s1[i * rp + c]);
        S2[o] = acc;
      }
    }
    // zero the pack padding of S2
    for (int o = Q + tid; o < round_up(Q, E); o += kThreads) S2[o] = czero<C>();
    __syncthreads();
  }

  // s3[alpha][b] = sum_q core[b][q] S2[alpha][q]; rows of both polarisations share the waves
  {
    const int rb0 = it0.rb, rb1 = it1.rb;
    wave_rowdots<T>(fac + it0.off_core, it0.ld_c, wave, rb0, kWaves, reinterpret_cast<const P*>(s2),
                    round_up(it0.rt * it0.rp, E) / E, s3, lane);
    // continue the round-robin where polarisation 0 left off
    const int first1 = ((wave - rb0) % kWaves + kWaves) % kWaves;
    wave_rowdots<T>(fac + it1.off_core, it1.ld_c, first1, rb1, kWaves, reinterpret_cast<const P*>(s2 + L.s2),
                    round_up(it1.rt * it1.rp, E) / E, s3 + L.s3, lane);
  }
  __syncthreads();

  // V[n] = conj(sum_alpha sum_b U^beta_alpha[n][b] s3[alpha][b])
  const int nb = it0.nb;
  const int npk = round_up(nb, E) / E;
  C* Vo = V + it0.row0 * nrhs + r;
  for (int base = 0; base < npk; base += kThreads * kColPacks) {
    P acc[kColPacks];
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) acc[j] = pzero<P>();
    block_colaxpy<T>(fac + it0.off_ubt, it0.ld_ub, it0.rb, s3, npk, base, tid, acc);
    block_colaxpy<T>(fac + it1.off_ubt, it1.ld_ub, it1.rb, s3 + L.s3, npk, base, tid, acc);
#pragma unroll
    for (int j = 0; j < kColPacks; ++j) {
      const int p = base + tid + kThreads * j;
      if (p < npk) {
        const C* vals = reinterpret_cast<const C*>(&acc[j]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int n = p * E + e;
          if (n < nb) Vo[(int64_t)n * nrhs] = conjc(vals[e]);
        }
      }
    }
  }
}

}  // namespace

template <typename T>
size_t tucker_agg_lds_bytes(const TuckMax& mx) {
  return AggLds<T>(mx).bytes();
}
template <typename T>
size_t tucker_disagg_lds_bytes(const TuckMax& mx) {
  return DisLds<T>(mx).bytes();
}

template <typename T>
hipError_t launch_tucker_agg(const void* fac, const TuckItem* items, const int32_t* order, int n_items,
                             const TuckMax& mx, int n_theta, int n_phi, int nrhs, const void* x, void* F,
                             hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_items == 0) return hipSuccess;
  const size_t lds = AggLds<T>(mx).bytes();
  dim3 grid(n_items, nrhs);
  hipLaunchKernelGGL(tucker_agg_kernel<T>, grid, dim3(kThreads), lds, s, static_cast<const C*>(fac), items,
                     order, mx, n_theta, n_phi, nrhs, static_cast<const C*>(x), static_cast<C*>(F));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tucker_disagg(const void* fac, const TuckItem* items, const int32_t* order, int n_groups,
                                const TuckMax& mx, int n_theta, int n_phi, int nrhs, const void* G, void* V,
                                hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_groups == 0) return hipSuccess;
  const size_t lds = DisLds<T>(mx).bytes();
  dim3 grid(n_groups, nrhs);
  hipLaunchKernelGGL(tucker_disagg_kernel<T>, grid, dim3(kThreads), lds, s, static_cast<const C*>(fac), items,
                     order, mx, n_theta, n_phi, nrhs, static_cast<const C*>(G), static_cast<C*>(V));
  return hipGetLastError();
}

template size_t tucker_agg_lds_bytes<float>(const TuckMax&);
template size_t tucker_agg_lds_bytes<double>(const TuckMax&);
template size_t tucker_disagg_lds_bytes<float>(const TuckMax&);
template size_t tucker_disagg_lds_bytes<double>(const TuckMax&);
template hipError_t launch_tucker_agg<float>(const void*, const TuckItem*, const int32_t*, int, const TuckMax&,
                                             int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_tucker_agg<double>(const void*, const TuckItem*, const int32_t*, int, const TuckMax&,
                                              int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_tucker_disagg<float>(const void*, const TuckItem*, const int32_t*, int,
                                                const TuckMax&, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_tucker_disagg<double>(const void*, const TuckItem*, const int32_t*, int,
                                                 const TuckMax&, int, int, int, const void*, void*, hipStream_t);

}  // namespace tuckfmm
