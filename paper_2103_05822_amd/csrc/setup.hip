// Setup kernels: the far-field signatures of eq. (4) and the data movement used by
// the HOSVD driver.  All FP64.
#include <hip/hip_runtime.h>
#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

// One workgroup per (basis row, 256 directions).  rowdata holds, for each of the
// six quadrature points of the two triangles, r_q - r_v and the RWG vector rho_q
// (r_q - p+ on T+, p- - r_q on T-), then l_n / 6 (3-point rule weight A/3 times
// the RWG normalisation l_n / (2A)).
__global__ __launch_bounds__(256) void farfield_fill_kernel(const double* __restrict__ rowdata,
                                                            const double* __restrict__ dirs, int ndir,
                                                            double k, double2* __restrict__ out) {
  const int64_t n = blockIdx.x;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= ndir) return;
  const double* rd = rowdata + n * kRowDoubles;
  const double* d = dirs + (int64_t)i * 9;
  const double kx = d[0], ky = d[1], kz = d[2];
  const double tx = d[3], ty = d[4], tz = d[5];
  const double px = d[6], py = d[7], pz = d[8];
  double2 at = make_double2(0.0, 0.0), ap = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double* e = rd + q * 6;
    const double ph = k * (e[0] * kx + e[1] * ky + e[2] * kz);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double wt = e[3] * tx + e[4] * ty + e[5] * tz;
    const double wp = e[3] * px + e[4] * py + e[5] * pz;
    at.x += wt * cs;
    at.y += wt * sn;
    ap.x += wp * cs;
    ap.y += wp * sn;
  }
  const double sc = rd[36];
  out[(n * 2 + 0) * ndir + i] = make_double2(sc * at.x, sc * at.y);
  out[(n * 2 + 1) * ndir + i] = make_double2(sc * ap.x, sc * ap.y);
}

// Plane-wave excitation, the right-hand side of eq. (2): one thread per (basis row n,
// wave r), x[n][r] = -(l_n / 6) sum_q (e_r . rho_q) exp(-j k k_r . r_q) over the six
// rule points of the row (rowdata as above; r_q = (r_q - r_v) + r_v with the row's
// box centre r_v in rowdata[37..39]).  waves: [nrhs][6] = k_hat, e_hat.
template <typename C>
__global__ __launch_bounds__(256) void planewave_kernel(const double* __restrict__ rowdata, int64_t rows,
                                                        const double* __restrict__ waves, int nrhs, double k,
                                                        C* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * nrhs) return;
  const int64_t n = e / nrhs;
  const int r = (int)(e - n * nrhs);
  const double* rd = rowdata + n * kRowDoubles;
  const double* w = waves + (int64_t)r * 6;
  const double kx = w[0], ky = w[1], kz = w[2];
  const double ex = w[3], ey = w[4], ez = w[5];
  const double base = rd[37] * kx + rd[38] * ky + rd[39] * kz;  // k_hat . r_v
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double* p = rd + q * 6;
    const double ph = -k * (base + p[0] * kx + p[1] * ky + p[2] * kz);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double a = p[3] * ex + p[4] * ey + p[5] * ez;
    re += a * cs;
    im += a * sn;
  }
  using R = decltype(C{}.x);
  const double sc = -rd[36];
  out[e] = C{(R)(sc * re), (R)(sc * im)};
}

// Copy one polarisation of a group's far-field rows into two contiguous slabs:
//   out_tp [nb][n_theta][n_phi]   and   out_pt [nb][n_phi][n_theta]
__global__ __launch_bounds__(256) void gather_slab_kernel(const double2* __restrict__ ff, int64_t row0, int nb,
                                                          int alpha, int n_theta, int n_phi,
                                                          double2* __restrict__ out_tp,
                                                          double2* __restrict__ out_pt) {
  const int ndir = n_theta * n_phi;
  const int64_t total = (int64_t)nb * ndir;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t n = e / ndir;
    const int i = (int)(e - n * ndir);
    const double2 v = ff[((row0 + n) * 2 + alpha) * ndir + i];
    out_tp[e] = v;
    if (out_pt) {
      const int it = i / n_phi, ip = i - it * n_phi;
      out_pt[n * ndir + (int64_t)ip * n_theta + it] = v;
    }
  }
}

// dst (column-major n x r) = columns n-1, n-2, ..., n-r of src (column-major n x n):
// eigenvectors returned in ascending eigenvalue order become descending.
__global__ __launch_bounds__(256) void select_cols_rev_kernel(const double2* __restrict__ src, int n, int r,
                                                              double2* __restrict__ dst) {
  const int64_t total = (int64_t)n * r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / n, i = e - j * n;
    dst[e] = src[(int64_t)(n - 1 - j) * n + i];
  }
}

// out[k] = sum_l |a[k sk + l sl]|^2 for k < K, l < L (FP64; one workgroup per k):
// the energy a tensor keeps along each candidate factor column.
__global__ __launch_bounds__(256) void strided_energy_kernel(const double2* __restrict__ a, int64_t sk, int64_t L,
                                                             int64_t sl, double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t k = blockIdx.x;
  double acc = 0.0;
  for (int64_t l = threadIdx.x; l < L; l += 256) {
    const double2 v = a[k * sk + l * sl];
    acc += v.x * v.x + v.y * v.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

// Gram matrices of the theta and phi unfoldings of one tensor held as a slab
// s [nb][nt][np] (one n_theta x n_phi block S_n per basis function):
//   Gt = sum_n S_n S_n^H  (nt x nt),   Gp = sum_n S_n^T conj(S_n)  (np x np).
// Stage 1: workgroup (c, y) sums rows n of chunk c for 4x4 output tiles
// y*512 .. y*512+511 (theta tiles first, then phi tiles) into part[c][.]
// (entries [0, nt*nt) column-major Gt, then [nt*nt, nt*nt + np*np) column-major Gp).
constexpr int kGramThreads = 512;
__global__ __launch_bounds__(kGramThreads) void mode_gram_partial_kernel(const double2* __restrict__ s, int nb,
                                                                         int nt, int np, int rows_per,
                                                                         double2* __restrict__ part) {
  extern __shared__ double2 slab[];  // nt * np
  const int c = blockIdx.x;
  const int n0 = c * rows_per, n1 = min(nb, n0 + rows_per);
  const int tnt = (nt + 3) / 4, tnp = (np + 3) / 4;
  const int tt = tnt * tnt, pt = tnp * tnp;
  const int task = blockIdx.y * kGramThreads + threadIdx.x;
  int kind = -1, bi = 0, bk = 0;
  if (task < tt) {
    kind = 0;
    bi = task / tnt;
    bk = task - bi * tnt;
  } else if (task < tt + pt) {
    kind = 1;
    bi = (task - tt) / tnp;
    bk = (task - tt) - bi * tnp;
  }
  double2 acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = make_double2(0.0, 0.0);
  const int nd = nt * np;
  for (int n = n0; n < n1; ++n) {
    __syncthreads();
    for (int e = threadIdx.x; e < nd; e += kGramThreads) slab[e] = s[(int64_t)n * nd + e];
    __syncthreads();
    if (kind == 0) {
      for (int j = 0; j < np; ++j) {
        double2 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = 4 * bi + u, k = 4 * bk + u;
          a[u] = i < nt ? slab[i * np + j] : make_double2(0.0, 0.0);
          b[u] = k < nt ? slab[k * np + j] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) cfma_conj(acc[u][v], b[v], a[u]);
      }
    } else if (kind == 1) {
      for (int i = 0; i < nt; ++i) {
        double2 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = 4 * bi + u, l = 4 * bk + u;
          a[u] = j < np ? slab[i * np + j] : make_double2(0.0, 0.0);
          b[u] = l < np ? slab[i * np + l] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) cfma_conj(acc[u][v], b[v], a[u]);
      }
    }
  }
  if (kind < 0) return;
  const int m = kind == 0 ? nt : np;
  double2* out = part + (int64_t)c * (nt * nt + np * np) + (kind == 0 ? 0 : nt * nt);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * bi + u, q = 4 * bk + v;
      if (r < m && q < m) out[r + (int64_t)q * m] = acc[u][v];  // column-major (r, q)
    }
}

// Stage 2: Gt / Gp = sum of the parts in chunk order (deterministic).
__global__ __launch_bounds__(256) void mode_gram_reduce_kernel(const double2* __restrict__ part, int nchunks,
                                                               int nt, int np, double2* __restrict__ gt,
                                                               double2* __restrict__ gp) {
  const int total = nt * nt + np * np;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int c = 0; c < nchunks; ++c) {
    const double2 v = part[(int64_t)c * total + e];
    acc.x += v.x;
    acc.y += v.y;
  }
  if (e < nt * nt) gt[e] = acc;
  else gp[e - nt * nt] = acc;
}

}  // namespace

int mode_gram_chunks(int nb) { return (nb + kGramRows - 1) / kGramRows; }

hipError_t launch_mode_gram(const void* slab, int nb, int nt, int np, void* part, void* gt, void* gp,
                            hipStream_t s) {
  const int nchunks = mode_gram_chunks(nb);
  const int tasks = ((nt + 3) / 4) * ((nt + 3) / 4) + ((np + 3) / 4) * ((np + 3) / 4);
  dim3 grid(nchunks, (tasks + kGramThreads - 1) / kGramThreads);
  const size_t lds = sizeof(double2) * (size_t)nt * np;
  hipLaunchKernelGGL(mode_gram_partial_kernel, grid, dim3(kGramThreads), lds, s,
                     static_cast<const double2*>(slab), nb, nt, np, kGramRows, static_cast<double2*>(part));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int total = nt * nt + np * np;
  hipLaunchKernelGGL(mode_gram_reduce_kernel, dim3((total + 255) / 256), dim3(256), 0, s,
                     static_cast<const double2*>(part), nchunks, nt, np, static_cast<double2*>(gt),
                     static_cast<double2*>(gp));
  return hipGetLastError();
}

hipError_t launch_select_cols_rev(const void* src, int n, int r, void* dst, hipStream_t s) {
  const int64_t total = (int64_t)n * r;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(select_cols_rev_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const double2*>(src), n, r, static_cast<double2*>(dst));
  return hipGetLastError();
}

hipError_t launch_strided_energy(const void* a, int K, int64_t sk, int64_t L, int64_t sl, double* out,
                                 hipStream_t s) {
  if (K <= 0) return hipSuccess;
  hipLaunchKernelGGL(strided_energy_kernel, dim3((unsigned)K), dim3(256), 0, s, static_cast<const double2*>(a), sk,
                     L, sl, out);
  return hipGetLastError();
}

hipError_t launch_farfield_fill(const double* rowdata, int64_t rows, const double* dirs, int ndir, double k,
                                void* out, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  dim3 grid((unsigned)rows, (ndir + 255) / 256);
  hipLaunchKernelGGL(farfield_fill_kernel, grid, dim3(256), 0, s, rowdata, dirs, ndir, k,
                     static_cast<double2*>(out));
  return hipGetLastError();
}

hipError_t launch_planewave(const double* rowdata, int64_t rows, const double* waves, int nrhs, double k,
                            size_t elem_bytes, void* out, hipStream_t s) {
  const int64_t total = rows * nrhs;
  if (total == 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (elem_bytes == 16)
    hipLaunchKernelGGL(planewave_kernel<double2>, grid, dim3(256), 0, s, rowdata, rows, waves, nrhs, k,
                       static_cast<double2*>(out));
  else if (elem_bytes == 8)
    hipLaunchKernelGGL(planewave_kernel<float2>, grid, dim3(256), 0, s, rowdata, rows, waves, nrhs, k,
                       static_cast<float2*>(out));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gather_slab(const void* farfield, int64_t row0, int nb, int alpha, int n_theta, int n_phi,
                              void* out_tp, void* out_pt, hipStream_t s) {
  const int64_t total = (int64_t)nb * n_theta * n_phi;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(gather_slab_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const double2*>(farfield), row0, nb, alpha, n_theta, n_phi,
                     static_cast<double2*>(out_tp), static_cast<double2*>(out_pt));
  return hipGetLastError();
}

}  // namespace tuckfmm
