// Dense (plain-method) aggregation and disaggregation, eqs. (3) and (5), Figs. 2(a)
// and 3(a).  Both kernels are pure HBM streams over the far-field array
// [N][2][N_dir] (a group's rows are contiguous):
//   aggregation    F[g][col] = sum_n A[n][col] x[n]      one thread per column,
//                                                         rows walked in order
//   disaggregation V[n] = sum_col conj(A[n][col]) G[g][col]   one wavefront per row,
//                                                         lane-strided, butterfly sum
#include <hip/hip_runtime.h>
#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kCols = 2;     // columns per thread in aggregation
constexpr int kRowUnroll = 4;

template <typename T>
__global__ __launch_bounds__(kThreads) void dense_agg_kernel(const typename Tr<T>::c* __restrict__ A,
                                                             const DenseGroup* __restrict__ groups, int n_chunks,
                                                             int ncols, int nrhs,
                                                             const typename Tr<T>::c* __restrict__ x,
                                                             typename Tr<T>::c* __restrict__ F) {
  using C = typename Tr<T>::c;
  const int g = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - g * n_chunks;
  const int r = blockIdx.y;
  const DenseGroup grp = groups[g];
  const int c0 = chunk * kThreads * kCols + threadIdx.x;
  bool in[kCols];
#pragma unroll
  for (int j = 0; j < kCols; ++j) in[j] = c0 + kThreads * j < ncols;
  C acc[kCols];
#pragma unroll
  for (int j = 0; j < kCols; ++j) acc[j] = czero<C>();
  const C* base = A + grp.row0 * ncols + c0;
  const C* xb = x + grp.row0 * nrhs + r;
  int n = 0;
  for (; n + kRowUnroll <= grp.nb; n += kRowUnroll) {
    C a[kRowUnroll][kCols];
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u)
#pragma unroll
      for (int j = 0; j < kCols; ++j)
        a[u][j] = in[j] ? base[(int64_t)(n + u) * ncols + kThreads * j] : czero<C>();
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) {
      const C xn = xb[(int64_t)(n + u) * nrhs];
#pragma unroll
      for (int j = 0; j < kCols; ++j) cfma(acc[j], a[u][j], xn);
    }
  }
  for (; n < grp.nb; ++n) {
    const C xn = xb[(int64_t)n * nrhs];
#pragma unroll
    for (int j = 0; j < kCols; ++j)
      if (in[j]) cfma(acc[j], base[(int64_t)n * ncols + kThreads * j], xn);
  }
#pragma unroll
  for (int j = 0; j < kCols; ++j)
    if (in[j]) F[((int64_t)g * ncols + c0 + kThreads * j) * nrhs + r] = acc[j];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void dense_disagg_kernel(const typename Tr<T>::c* __restrict__ A,
                                                                const int64_t* __restrict__ offsets,
                                                                int n_groups, int64_t n_rows, int ncols,
                                                                int nrhs,
                                                                const typename Tr<T>::c* __restrict__ Gin,
                                                                typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int r = blockIdx.y;
  if (n >= n_rows) return;  // no barrier below
  // group of row n: largest g with offsets[g] <= n
  int lo = 0, hi = n_groups;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offsets[mid] <= n) lo = mid; else hi = mid;
  }
  const C* row = A + n * ncols;
  const C* gv = Gin + (int64_t)lo * ncols * nrhs + r;
  C a0 = czero<C>(), a1 = czero<C>(), a2 = czero<C>(), a3 = czero<C>();
  int c = lane;
  for (; c + 192 < ncols; c += 256) {
    const C u0 = row[c], u1 = row[c + 64], u2 = row[c + 128], u3 = row[c + 192];
    const C g0 = gv[(int64_t)c * nrhs], g1 = gv[(int64_t)(c + 64) * nrhs];
    const C g2 = gv[(int64_t)(c + 128) * nrhs], g3 = gv[(int64_t)(c + 192) * nrhs];
    cfma_conj(a0, u0, g0);
    cfma_conj(a1, u1, g1);
    cfma_conj(a2, u2, g2);
    cfma_conj(a3, u3, g3);
  }
  for (; c < ncols; c += 64) cfma_conj(a0, row[c], gv[(int64_t)c * nrhs]);
  a0.x += a1.x + a2.x + a3.x;
  a0.y += a1.y + a2.y + a3.y;
  a0 = wave_sum(a0);
  if (lane == 0) V[n * nrhs + r] = a0;
}

}  // namespace

template <typename T>
hipError_t launch_dense_agg(const void* A, const DenseGroup* groups, int n_groups, int ncols, int nrhs,
                            const void* x, void* F, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_groups == 0) return hipSuccess;
  const int n_chunks = (ncols + kThreads * kCols - 1) / (kThreads * kCols);
  dim3 grid((unsigned)n_groups * n_chunks, nrhs);
  hipLaunchKernelGGL(dense_agg_kernel<T>, grid, dim3(kThreads), 0, s, static_cast<const C*>(A), groups, n_chunks,
                     ncols, nrhs, static_cast<const C*>(x), static_cast<C*>(F));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_disagg(const void* A, const int64_t* offsets, int n_groups, int64_t n_rows, int ncols,
                               int nrhs, const void* G, void* V, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_rows == 0) return hipSuccess;
  const int64_t blocks = (n_rows + kThreads / 64 - 1) / (kThreads / 64);
  dim3 grid((unsigned)blocks, nrhs);
  hipLaunchKernelGGL(dense_disagg_kernel<T>, grid, dim3(kThreads), 0, s, static_cast<const C*>(A), offsets,
                     n_groups, n_rows, ncols, nrhs, static_cast<const C*>(G), static_cast<C*>(V));
  return hipGetLastError();
}

template hipError_t launch_dense_agg<float>(const void*, const DenseGroup*, int, int, int, const void*, void*,
                                            hipStream_t);
template hipError_t launch_dense_agg<double>(const void*, const DenseGroup*, int, int, int, const void*, void*,
                                             hipStream_t);
template hipError_t launch_dense_disagg<float>(const void*, const int64_t*, int, int64_t, int, int, const void*,
                                               void*, hipStream_t);
template hipError_t launch_dense_disagg<double>(const void*, const int64_t*, int, int64_t, int, int, const void*,
                                                void*, hipStream_t);

}  // namespace tuckfmm
