// Dense (plain-method) aggregation and disaggregation, eqs. (3) and (5), Figs. 2(a)
// and 3(a).  Both kernels are pure HBM streams over the far-field array
// [N][2][N_dir] (a group's rows are contiguous):
//   aggregation    F[g][col] = sum_n A[n][col] x[n]      one thread per column,
//                                                         rows walked in order
//   disaggregation V[n] = sum_col conj(A[n][col]) G[g][col]   one wavefront per row,
//                                                         lane-strided, butterfly sum
// with up to 8 right-hand sides per read of A.  With 2 or more right-hand sides the
// disaggregation works on blocks of rows of one group instead (see
// dense_disagg_block_kernel).
#include <hip/hip_runtime.h>
#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kCols = 2;     // columns per thread in aggregation

// Right-hand sides are taken RB at a time (blockIdx.y walks the blocks of RB): every
// element of A read from HBM serves RB right-hand sides, so a pass over R <= 8 of
// them reads A once.  nr = min(RB, nrhs - r0) of a block's RB columns are valid.

template <typename T, int RB>
__global__ __launch_bounds__(kThreads) void dense_agg_kernel(const typename Tr<T>::c* __restrict__ A,
                                                             const DenseGroup* __restrict__ groups, int n_chunks,
                                                             int ncols, int nrhs,
                                                             const typename Tr<T>::c* __restrict__ x,
                                                             typename Tr<T>::c* __restrict__ F) {
  using C = typename Tr<T>::c;
  // rows per iteration: the x values of a row are uniform across the workgroup and
  // live in scalar registers, RB of them per row
  constexpr int kRowUnroll = RB >= 4 ? 2 : 4;
  const int g = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - g * n_chunks;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const DenseGroup grp = groups[g];
  const int c0 = chunk * kThreads * kCols + threadIdx.x;
  bool in[kCols];
#pragma unroll
  for (int j = 0; j < kCols; ++j) in[j] = c0 + kThreads * j < ncols;
  C acc[kCols][RB];
#pragma unroll
  for (int j = 0; j < kCols; ++j)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[j][r] = czero<C>();
  const C* base = A + grp.row0 * ncols + c0;
  const C* xb = x + grp.row0 * nrhs + r0;
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
      C xn[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) xn[r] = r < nr ? xb[(int64_t)(n + u) * nrhs + r] : czero<C>();
#pragma unroll
      for (int j = 0; j < kCols; ++j)
#pragma unroll
        for (int r = 0; r < RB; ++r) cfma(acc[j][r], a[u][j], xn[r]);
    }
  }
  for (; n < grp.nb; ++n) {
    C xn[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) xn[r] = r < nr ? xb[(int64_t)n * nrhs + r] : czero<C>();
#pragma unroll
    for (int j = 0; j < kCols; ++j) {
      const C a = in[j] ? base[(int64_t)n * ncols + kThreads * j] : czero<C>();
#pragma unroll
      for (int r = 0; r < RB; ++r) cfma(acc[j][r], a, xn[r]);
    }
  }
#pragma unroll
  for (int j = 0; j < kCols; ++j)
    if (in[j]) {
      C* out = F + ((int64_t)g * ncols + c0 + kThreads * j) * nrhs + r0;
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < nr) out[r] = acc[j][r];
    }
}

// Disaggregation with one right-hand side: a wavefront per row, four columns in
// flight per lane, butterfly sum.
template <typename T>
__global__ __launch_bounds__(kThreads) void dense_disagg_kernel(const typename Tr<T>::c* __restrict__ A,
                                                                const int64_t* __restrict__ offsets,
                                                                int n_groups, int64_t n_rows, int ncols,
                                                                const typename Tr<T>::c* __restrict__ Gin,
                                                                typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  constexpr int U = 4;  // columns in flight per lane
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (n >= n_rows) return;  // no barrier below
  // group of row n: largest g with offsets[g] <= n
  int lo = 0, hi = n_groups;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offsets[mid] <= n) lo = mid; else hi = mid;
  }
  const C* row = A + n * ncols;
  const C* gv = Gin + (int64_t)lo * ncols;
  C acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = czero<C>();
  int c = lane;
  for (; c + 64 * (U - 1) < ncols; c += 64 * U) {
    C a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = row[c + 64 * u];
#pragma unroll
    for (int u = 0; u < U; ++u) cfma_conj(acc[u], a[u], gv[c + 64 * u]);
  }
  for (; c < ncols; c += 64) cfma_conj(acc[0], row[c], gv[c]);
  C s = acc[0];
#pragma unroll
  for (int u = 1; u < U; ++u) {
    s.x += acc[u].x;
    s.y += acc[u].y;
  }
  s = wave_sum(s);
  if (lane == 0) V[n] = s;
}

// Disaggregation with RB = 2, 4 or 8 right-hand sides per read of A, over the row
// blocks of the plan (up to 16 rows of one group).  Read per row, the group's G would
// cost RB times the row's bytes, and a lane's RB values of one column sit 16 RB bytes
// apart from the next lane's, so each load instruction would touch 64 cache lines.
// Instead the workgroup walks the columns in chunks of 64: its 256 threads load the
// chunk's G[g][c][r0 .. r0 + RB) with coalesced loads into LDS (double buffered, one
// barrier per chunk), and wavefront w, owning rows 4w .. 4w + 3 of the block, reads a
// lane's column from there for its four rows while the rows of A stream from HBM
// (prefetched one chunk ahead).  The plan orders the blocks so that each XCD works on
// a few groups at a time, whose G then stays in its L2.
template <typename T, int RB>
__global__ __launch_bounds__(kThreads) void dense_disagg_block_kernel(const typename Tr<T>::c* __restrict__ A,
                                                                      const DenseBlock* __restrict__ blocks,
                                                                      int ncols, int nrhs,
                                                                      const typename Tr<T>::c* __restrict__ Gin,
                                                                      typename Tr<T>::c* __restrict__ V) {
  using C = typename Tr<T>::c;
  constexpr int RW = 4;                               // rows per wavefront
  constexpr int CW = 64;                              // columns per chunk
  constexpr int GS = RB + 1;                          // LDS row stride (complex): spreads the banks
  constexpr int GL = (CW * RB + kThreads - 1) / kThreads;  // G elements per thread and chunk
  __shared__ C gsh[2][CW * GS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const DenseBlock b = blocks[blockIdx.x];
  const int i0 = RW * w;
  const int nrow = max(0, min(RW, b.rows - i0));  // uniform per wavefront; 0: loads and barriers only
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const C* rows = A + (b.row0 + min(i0, b.rows - 1)) * ncols;
  const C* gv = Gin + (int64_t)b.group * ncols * nrhs + r0;
  const int nchunks = (ncols + CW - 1) / CW;

  C greg[GL];
  auto load_g = [&](int chunk) {
#pragma unroll
    for (int k = 0; k < GL; ++k) {
      const int e = tid + kThreads * k, cc = e / RB, r = e % RB, c = chunk * CW + cc;
      greg[k] = e < CW * RB && c < ncols && r < nr ? gv[(int64_t)c * nrhs + r] : czero<C>();
    }
  };
  auto store_g = [&](int buf) {
#pragma unroll
    for (int k = 0; k < GL; ++k) {
      const int e = tid + kThreads * k;
      if (e < CW * RB) gsh[buf][(e / RB) * GS + e % RB] = greg[k];
    }
  };
  auto load_a = [&](int chunk, C (&a)[RW]) {
    const int c = chunk * CW + lane;
#pragma unroll
    for (int i = 0; i < RW; ++i) a[i] = i < nrow && c < ncols ? rows[(int64_t)i * ncols + c] : czero<C>();
  };

  C acc[RW][RB];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[i][r] = czero<C>();
  C a[RW], an[RW];
  load_g(0);
  load_a(0, a);
  store_g(0);
  __syncthreads();
  for (int chunk = 0; chunk < nchunks; ++chunk) {
    const bool more = chunk + 1 < nchunks;
    if (more) {
      load_a(chunk + 1, an);
      load_g(chunk + 1);
    }
    const C* gc = &gsh[chunk & 1][lane * GS];
    C gt[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) gt[r] = gc[r];
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
      for (int r = 0; r < RB; ++r) cfma_conj(acc[i][r], a[i], gt[r]);
    if (more) {
      store_g((chunk + 1) & 1);  // that buffer was last read before the previous barrier
#pragma unroll
      for (int i = 0; i < RW; ++i) a[i] = an[i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    if (i >= nrow) break;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const C sum = wave_sum(acc[i][r]);
      if (lane == 0 && r < nr) V[(b.row0 + i0 + i) * nrhs + r0 + r] = sum;
    }
  }
}

// RB for a call: the smallest of 1, 2, 4, 8 covering nrhs (8 beyond).
int rhs_block(int nrhs) { return nrhs >= 8 ? 8 : (nrhs > 2 ? 4 : nrhs); }

}  // namespace

#define TFMM_RB_SWITCH(rb, ...) \
  switch (rb) {                  \
    case 1: {                    \
      constexpr int RB = 1;      \
      __VA_ARGS__;               \
      break;                     \
    }                            \
    case 2: {                    \
      constexpr int RB = 2;      \
      __VA_ARGS__;               \
      break;                     \
    }                            \
    case 4: {                    \
      constexpr int RB = 4;      \
      __VA_ARGS__;               \
      break;                     \
    }                            \
    default: {                   \
      constexpr int RB = 8;      \
      __VA_ARGS__;               \
      break;                     \
    }                            \
  }

template <typename T>
hipError_t launch_dense_agg(const void* A, const DenseGroup* groups, int n_groups, int ncols, int nrhs,
                            const void* x, void* F, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_groups == 0) return hipSuccess;
  const int n_chunks = (ncols + kThreads * kCols - 1) / (kThreads * kCols);
  const int rb = rhs_block(nrhs);
  dim3 grid((unsigned)n_groups * n_chunks, (nrhs + rb - 1) / rb);
  TFMM_RB_SWITCH(rb, hipLaunchKernelGGL((dense_agg_kernel<T, RB>), grid, dim3(kThreads), 0, s,
                                        static_cast<const C*>(A), groups, n_chunks, ncols, nrhs,
                                        static_cast<const C*>(x), static_cast<C*>(F)))
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_disagg(const void* A, const int64_t* offsets, int n_groups, int64_t n_rows,
                               const DenseBlock* row_blocks, int n_blocks, int ncols, int nrhs, const void* G,
                               void* V, hipStream_t s) {
  using C = typename Tr<T>::c;
  if (n_rows == 0) return hipSuccess;
  const int rb = rhs_block(nrhs);
  if (rb == 1) {
    const int64_t blocks = (n_rows + kThreads / 64 - 1) / (kThreads / 64);
    hipLaunchKernelGGL((dense_disagg_kernel<T>), dim3((unsigned)blocks), dim3(kThreads), 0, s,
                       static_cast<const C*>(A), offsets, n_groups, n_rows, ncols, static_cast<const C*>(G),
                       static_cast<C*>(V));
    return hipGetLastError();
  }
  if (n_blocks <= 0 || row_blocks == nullptr) return hipErrorInvalidValue;
  dim3 grid((unsigned)n_blocks, (nrhs + rb - 1) / rb);
  TFMM_RB_SWITCH(rb, hipLaunchKernelGGL((dense_disagg_block_kernel<T, RB>), grid, dim3(kThreads), 0, s,
                                        static_cast<const C*>(A), row_blocks, ncols, nrhs,
                                        static_cast<const C*>(G), static_cast<C*>(V)))
  return hipGetLastError();
}

template hipError_t launch_dense_agg<float>(const void*, const DenseGroup*, int, int, int, const void*, void*,
                                            hipStream_t);
template hipError_t launch_dense_agg<double>(const void*, const DenseGroup*, int, int, int, const void*, void*,
                                             hipStream_t);
template hipError_t launch_dense_disagg<float>(const void*, const int64_t*, int, int64_t, const DenseBlock*, int,
                                               int, int, const void*, void*, hipStream_t);
template hipError_t launch_dense_disagg<double>(const void*, const int64_t*, int, int64_t, const DenseBlock*, int,
                                                int, int, const void*, void*, hipStream_t);

}  // namespace tuckfmm
