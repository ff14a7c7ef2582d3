// Multi-right-hand-side Tucker aggregation and disaggregation on the matrix cores.
//
// With R right-hand sides every contraction of Section II.C becomes a matrix product
// (Fig. 2(b) and Fig. 3(b) applied to R columns at once).  Each stage is four
// launches of one grouped complex GEMM kernel; launch j computes contraction j of
// every (group, polarisation) item, with intermediates in scratch memory:
//   aggregation    Y = U^beta^T X,  T = core^T Y,  then U^theta / U^phi on T
//   disaggregation the U^theta / U^phi products on conj(G), s = core S,
//                  V += conj(U^beta s)
// The descriptors of the products are built on the host (mrhs_plan.cpp); this file
// holds the kernel.  One launch may mix products of both stages (a pass).
//
// A complex product C = A B runs on real MFMA instructions through the identity
//   [Re C, Im C] = [Re A, Im A] [[Re B, Im B], [-Im B, Re B]]
// with A read as a real matrix whose columns interleave (Re, Im) -- the stored
// layout -- and B expanded on the fly: no arithmetic is wasted (8 real flops per
// complex multiply-add).  Workgroup tile: 64 rows x 32 complex columns, K in steps of
// 16 complex values, operands staged through LDS (double buffered), four wavefronts
// each owning 16 rows x 64 real columns = four 16x16 MFMA accumulators.
//
// Arithmetic variants (factors are stored as complex64 in every variant):
//   0  FP32    v_mfma_f32_16x16x4_f32 on the FP32 operands;
//   1  BF16x2  v_mfma_f32_16x16x32_bf16; both operands are split into bf16 pieces
//              v = hi + lo while they are read from LDS, and each product accumulates
//              hi*hi + hi*lo + lo*hi in FP32 (the dropped terms are below 2^-16
//              relative);
//   2  BF16x3  three pieces v = hi + mid + lo and the six products whose order is at
//              most 2^-16 (hi*hi, hi*mid, mid*hi, hi*lo, mid*mid, lo*hi): FP32-level
//              accuracy at six bf16 instructions per step.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMT = 256;  // threads
constexpr int kBM = 64;   // rows per tile
constexpr int kBN = 32;   // complex columns per tile
constexpr int kKC = 16;   // complex K per step
constexpr int kAS = kKC + 2;  // LDS row stride of A (complex), keeps 16-byte alignment
constexpr int kBS = kBN + 2;  // LDS row stride of B (complex)

__device__ __forceinline__ int64_t col_off(int n, int ni, int shi) { return (int64_t)(n / ni) * shi + n % ni; }

// -------------------------------------------------------------------- staging
// Global -> registers for one K step: A tile (kBM x kKC complex), B tile (kKC x kBN).
struct Stage {
  float4 a[2];  // two complex pairs of A per thread
  float4 b;     // one complex pair of B per thread
};

__device__ __forceinline__ float2 cj(float2 v, bool c) { return c ? make_float2(v.x, -v.y) : v; }

__device__ __forceinline__ void load_stage(const CGemm& p, const float2* A, const float2* B, int m0, int n0, int k0,
                                           int tid, Stage& st) {
  const bool ca = p.flags & kConjA, cb = p.flags & kConjB;
  // 16-byte loads need an even complex offset for every pair
  const bool avec = !((p.a | (p.lda_k == 1 ? p.lda_m : p.lda_k)) & 1);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;  // pair index 0..511
    float2 v0 = make_float2(0.f, 0.f), v1 = v0;
    if (p.lda_k == 1) {  // K contiguous: pair = (m, 2kp), (m, 2kp + 1)
      const int m = m0 + pr / 8, k = k0 + 2 * (pr % 8);
      if (m < p.M) {
        const float2* src = A + p.a + (int64_t)m * p.lda_m + k;
        if (k + 1 < p.K && avec) {
          const float4 q = *reinterpret_cast<const float4*>(src);
          v0 = make_float2(q.x, q.y);
          v1 = make_float2(q.z, q.w);
        } else {
          if (k < p.K) v0 = src[0];
          if (k + 1 < p.K) v1 = src[1];
        }
      }
    } else {  // M contiguous: pair = (2mp, k), (2mp + 1, k)
      const int k = k0 + pr / 32, m = m0 + 2 * (pr % 32);
      if (k < p.K) {
        const float2* src = A + p.a + m + (int64_t)k * p.lda_k;
        if (m + 1 < p.M && avec) {
          const float4 q = *reinterpret_cast<const float4*>(src);
          v0 = make_float2(q.x, q.y);
          v1 = make_float2(q.z, q.w);
        } else {
          if (m < p.M) v0 = src[0];
          if (m + 1 < p.M) v1 = src[1];
        }
      }
    }
    v0 = cj(v0, ca);
    v1 = cj(v1, ca);
    st.a[j] = make_float4(v0.x, v0.y, v1.x, v1.y);
  }
  {
    const int k = k0 + tid / 16, n = n0 + 2 * (tid % 16);
    float2 v0 = make_float2(0.f, 0.f), v1 = v0;
    if (k < p.K && n < p.N) {  // N and the column blocks are even: the pair never splits
      const float4 q =
          *reinterpret_cast<const float4*>(B + p.b + (int64_t)k * p.ldb_k + col_off(n, p.b_ni, p.b_shi));
      v0 = cj(make_float2(q.x, q.y), cb);
      v1 = cj(make_float2(q.z, q.w), cb);
    }
    st.b = make_float4(v0.x, v0.y, v1.x, v1.y);
  }
}

// Registers -> LDS.  A as [kBM][kAS] complex, B as [kKC][kBS] complex.
__device__ __forceinline__ void store_stage(const CGemm& p, const Stage& st, float2* As, float2* Bs, int tid) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;
    if (p.lda_k == 1) {
      const int m = pr / 8, k = 2 * (pr % 8);
      *reinterpret_cast<float4*>(As + m * kAS + k) = st.a[j];
    } else {
      const int k = pr / 32, m = 2 * (pr % 32);
      As[m * kAS + k] = make_float2(st.a[j].x, st.a[j].y);
      As[(m + 1) * kAS + k] = make_float2(st.a[j].z, st.a[j].w);
    }
  }
  const int k = tid / 16, n = 2 * (tid % 16);
  *reinterpret_cast<float4*>(Bs + k * kBS + n) = st.b;
}

// ------------------------------------------------------------------- compute

// One K step on FP32 MFMA.  Lane (mi, kb) of wavefront w: rows 16w + mi; the real K
// index covered by instruction (h, s) is 16h + 4kb + s (a permutation of the step's
// 32 real indices, applied identically to A and B).
__device__ __forceinline__ void mma_step_f32(const float2* As, const float2* Bs, int w, int lane,
                                             floatx4 (&acc)[4]) {
  const int mi = lane % 16, kb = lane / 16;
  const int q = mi & 1;  // as a B column lane: real column parity (0: Re, 1: Im)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float4 a = *reinterpret_cast<const float4*>(As + (16 * w + mi) * kAS + 8 * h + 2 * kb);
    const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int nc = 8 * t + mi / 2;
      const float2 b0 = Bs[(8 * h + 2 * kb) * kBS + nc];
      const float2 b1 = Bs[(8 * h + 2 * kb + 1) * kBS + nc];
      // expanded B rows 2k (Re A) and 2k + 1 (Im A) at real column 2n + q
      const float bv[4] = {q ? b0.y : b0.x, q ? b0.x : -b0.y, q ? b1.y : b1.x, q ? b1.x : -b1.y};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc[t], 0, 0, 0);
    }
  }
}

// One K step on BF16 MFMA with operands split into NP pieces (2 or 3).  Lane (mi, kb)
// supplies the real K indices 8kb .. 8kb + 7 of the 32-wide instruction.
template <int NP>
__device__ __forceinline__ void split_bf16(float v, __bf16 (&pc)[NP]) {
  pc[0] = (__bf16)v;
  float r = v - (float)pc[0];
  pc[1] = (__bf16)r;
  if constexpr (NP == 3) {
    r -= (float)pc[1];
    pc[2] = (__bf16)r;
  }
}

template <int NP>
__device__ __forceinline__ void mma_step_bf16(const float2* As, const float2* Bs, int w, int lane,
                                              floatx4 (&acc)[4]) {
  const int mi = lane % 16, kb = lane / 16;
  const int q = mi & 1;
  bf16x8 ap[NP];
  {
    const float4 a0 = *reinterpret_cast<const float4*>(As + (16 * w + mi) * kAS + 4 * kb);
    const float4 a1 = *reinterpret_cast<const float4*>(As + (16 * w + mi) * kAS + 4 * kb + 2);
    const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 pc[NP];
      split_bf16<NP>(av[e], pc);
#pragma unroll
      for (int u = 0; u < NP; ++u) ap[u][e] = pc[u];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int nc = 8 * t + mi / 2;
    bf16x8 bp[NP];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float2 b = Bs[(4 * kb + e) * kBS + nc];
      // expanded B rows 2k (Re A) and 2k + 1 (Im A) at real column 2n + q
      const float v0 = q ? b.y : b.x, v1 = q ? b.x : -b.y;
      __bf16 p0[NP], p1[NP];
      split_bf16<NP>(v0, p0);
      split_bf16<NP>(v1, p1);
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        bp[u][2 * e] = p0[u];
        bp[u][2 * e + 1] = p1[u];
      }
    }
    // smallest terms first
    if constexpr (NP == 3) {
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[2], bp[0], acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], bp[1], acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], bp[2], acc[t], 0, 0, 0);
    }
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], bp[0], acc[t], 0, 0, 0);
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], bp[1], acc[t], 0, 0, 0);
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], bp[0], acc[t], 0, 0, 0);
  }
}

// ------------------------------------------------------------------- kernel

__device__ __forceinline__ float2* base_ptr(const CGemmBases& b, int i) {
  // i is uniform across the workgroup: a select chain, no indexed private array
  void* p = i == 0 ? b.p[0] : i == 1 ? b.p[1] : i == 2 ? b.p[2] : i == 3 ? b.p[3] : i == 4 ? b.p[4] : b.p[5];
  return static_cast<float2*>(p);
}

template <int VARIANT>
__global__ __launch_bounds__(kMT) void cgemm_kernel(const CGemm* __restrict__ probs, const CTile* __restrict__ tiles,
                                                    CGemmBases bases) {
  __shared__ __align__(16) float2 As[2][kBM * kAS];
  __shared__ __align__(16) float2 Bs[2][kKC * kBS];
  const CTile tl = tiles[blockIdx.x];
  const CGemm p = probs[tl.prob];
  const float2* A = base_ptr(bases, p.abase);
  const float2* B = base_ptr(bases, p.bbase);
  float2* Cp = base_ptr(bases, p.cbase);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nsteps = (p.K + kKC - 1) / kKC;

  for (int n0 = tl.n0; n0 < tl.n1; n0 += kBN) {
    floatx4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    Stage st;
    load_stage(p, A, B, tl.m0, n0, 0, tid, st);
    __syncthreads();  // previous column block finished reading LDS
    store_stage(p, st, As[0], Bs[0], tid);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
      const int cur = s & 1;
      if (s + 1 < nsteps) load_stage(p, A, B, tl.m0, n0, (s + 1) * kKC, tid, st);
      if constexpr (VARIANT == 0)
        mma_step_f32(As[cur], Bs[cur], w, lane, acc);
      else
        mma_step_bf16<VARIANT + 1>(As[cur], Bs[cur], w, lane, acc);
      if (s + 1 < nsteps) store_stage(p, st, As[cur ^ 1], Bs[cur ^ 1], tid);
      __syncthreads();
    }
    // epilogue: lane (ni, g) holds real rows 4g + i, real column 16t + ni
    const int ni = lane % 16, g = lane / 16;
    const int q = ni & 1;
    const bool conj_out = p.flags & kConjC, atomic = p.flags & kAtomicC;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = n0 + 8 * t + ni / 2;
      if (n >= p.N) continue;
      const int64_t coff = p.c + col_off(n, p.c_ni, p.c_shi);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = tl.m0 + 16 * w + 4 * g + i;
        if (m >= p.M) continue;
        float v = acc[t][i];
        if (conj_out && q) v = -v;
        float* dst = reinterpret_cast<float*>(Cp + coff + (int64_t)m * p.ldc_m) + q;
        if (atomic)
          atomicAdd(dst, v);
        else
          *dst = v;
      }
    }
  }
}

template <typename C>
__global__ __launch_bounds__(256) void mrhs_zero_kernel(C* __restrict__ v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v[i] = czero<C>();
}

}  // namespace

hipError_t launch_cgemm(int variant, const CGemm* probs, const CTile* tiles, int n_tiles, const CGemmBases& b,
                        hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (variant == 0)
    hipLaunchKernelGGL(cgemm_kernel<0>, dim3(n_tiles), dim3(kMT), 0, s, probs, tiles, b);
  else if (variant == 1)
    hipLaunchKernelGGL(cgemm_kernel<1>, dim3(n_tiles), dim3(kMT), 0, s, probs, tiles, b);
  else if (variant == 2)
    hipLaunchKernelGGL(cgemm_kernel<2>, dim3(n_tiles), dim3(kMT), 0, s, probs, tiles, b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_zero_c64(void* v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(mrhs_zero_kernel<float2>, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<float2*>(v), n);
  return hipGetLastError();
}

}  // namespace tuckfmm
