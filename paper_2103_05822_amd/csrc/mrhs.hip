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
// layout -- and B expanded to the 2 x 2 real blocks: no arithmetic is wasted (8 real
// flops per complex multiply-add).
//
// Workgroup tile: 64 rows x 64 complex columns (128 real), K in steps of 16 complex
// values (32 real).  Four wavefronts, each owning 16 rows x 128 real columns = eight
// 16 x 16 MFMA accumulators.  A workgroup walks its column blocks and K steps as one
// flat pipeline: the global loads of step s + 1 are in flight while step s runs on the
// matrix cores from LDS (double buffered); conjugation, B expansion and the bf16
// split happen when a step is written to LDS.
//
// Arithmetic variants (factors are stored as complex64 in every variant):
//   0  FP32    v_mfma_f32_16x16x4_f32 on the FP32 operands;
//   1  BF16x2  v_mfma_f32_16x16x32_bf16; both operands are split into bf16 pieces
//              v = hi + lo and each product accumulates hi*hi + hi*lo + lo*hi in FP32
//              (the dropped lo*lo term is below 2^-16 relative);
//   2  BF16x3  three pieces v = hi + mid + lo and the six products whose order is at
//              most 2^-16 (hi*hi, hi*mid, mid*hi, hi*lo, mid*mid, lo*hi): FP32-level
//              accuracy at six bf16 instructions per product.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kMT = 256;           // threads
constexpr int kBM = 64;            // rows per tile
constexpr int kBN = 64;            // complex columns per block
constexpr int kKC = 16;            // complex K per step
constexpr int kKR = 2 * kKC;       // real K per step
constexpr int kNT = 2 * kBN / 16;  // 16-column accumulators per wavefront (8)
// FP32 LDS strides (complex): padding keeps 16-byte alignment and spreads banks
constexpr int kAS = kKC + 2;
constexpr int kBS = kBN + 2;

__device__ __forceinline__ int64_t col_off(int n, int ni, int shi) { return (int64_t)(n / ni) * shi + n % ni; }

__device__ __forceinline__ float2* base_ptr(const CGemmBases& b, int i) {
  // i is uniform across the workgroup: a select chain, no indexed private array
  void* p = i == 0 ? b.p[0] : i == 1 ? b.p[1] : i == 2 ? b.p[2] : i == 3 ? b.p[3] : i == 4 ? b.p[4] : b.p[5];
  return static_cast<float2*>(p);
}

// ------------------------------------------------------------------ global loads
// One K step of raw operands in registers: two complex pairs of A and two of B per
// thread, plus validity bits.  Every load is unconditional (an invalid element reads
// the operand's first element instead) and nothing consumes the loaded values before
// the step is written to LDS, so the loads stay in flight while the previous step
// runs on the matrix cores.  AVEC (uniform per product): A pairs are loaded as one
// 16-byte access; the second element of a pair at the K (or M) tail then lies in the
// zero padding of the factor row (rows are padded to an even length), and is masked.
struct Stage {
  float4 a[2];
  float4 b[2];
  uint32_t ok;  // bits 0-3: A halves (pair j: bits 2j, 2j+1); bits 4-5: B pairs
};

template <bool AVEC>
__device__ __forceinline__ void load_stage(const CGemm& p, const float2* A, const float2* B, int m0, int n0, int k0,
                                           int tid, Stage& st) {
  uint32_t ok = 0;
  const float2* a0 = A + p.a;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;  // pair index 0..511
    bool ok0, ok1;
    int64_t i0, i1;
    if (p.lda_k == 1) {  // K contiguous: pair = (m, k), (m, k + 1)
      const int m = m0 + pr / 8, k = k0 + 2 * (pr % 8);
      ok0 = m < p.M && k < p.K;
      ok1 = m < p.M && k + 1 < p.K;
      i0 = (int64_t)m * p.lda_m + k;
      i1 = i0 + 1;
    } else {  // M contiguous: pair = (m, k), (m + 1, k)
      const int k = k0 + pr / 32, m = m0 + 2 * (pr % 32);
      ok0 = k < p.K && m < p.M;
      ok1 = k < p.K && m + 1 < p.M;
      i0 = m + (int64_t)k * p.lda_k;
      i1 = i0 + 1;
    }
    if constexpr (AVEC) {
      st.a[j] = *reinterpret_cast<const float4*>(a0 + (ok0 ? i0 : 0));
    } else {
      const float2 u0 = a0[ok0 ? i0 : 0];
      const float2 u1 = a0[ok1 ? i1 : 0];
      st.a[j] = make_float4(u0.x, u0.y, u1.x, u1.y);
    }
    ok |= (ok0 ? 1u : 0u) << (2 * j);
    ok |= (ok1 ? 1u : 0u) << (2 * j + 1);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;
    const int k = k0 + pr / 32, n = n0 + 2 * (pr % 32);
    const bool okb = k < p.K && n < p.N;  // N and the column blocks are even: a pair never splits
    const int64_t ib = okb ? (int64_t)k * p.ldb_k + col_off(n, p.b_ni, p.b_shi) : 0;
    st.b[j] = *reinterpret_cast<const float4*>(B + p.b + ib);
    ok |= (okb ? 1u : 0u) << (4 + j);
  }
  st.ok = ok;
}

// Operand values of a stage with the invalid elements zeroed and the conjugation
// flags applied (this is where the loads are waited for).
__device__ __forceinline__ float4 a_val(const CGemm& p, const Stage& st, int j) {
  float4 v = st.a[j];
  if (!(st.ok & (1u << (2 * j)))) v.x = v.y = 0.f;
  if (!(st.ok & (1u << (2 * j + 1)))) v.z = v.w = 0.f;
  if (p.flags & kConjA) {
    v.y = -v.y;
    v.w = -v.w;
  }
  return v;
}

__device__ __forceinline__ float4 b_val(const CGemm& p, const Stage& st, int j) {
  float4 v = st.b[j];
  if (!(st.ok & (1u << (4 + j)))) v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (p.flags & kConjB) {
    v.y = -v.y;
    v.w = -v.w;
  }
  return v;
}

// ------------------------------------------------------------------- FP32 variant
struct LdsF32 {
  float2 a[2][kBM * kAS];
  float2 b[2][kKC * kBS];
};

__device__ __forceinline__ void store_f32(const CGemm& p, const Stage& st, LdsF32& L, int buf, int tid) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;
    const float4 v = a_val(p, st, j);
    if (p.lda_k == 1) {
      const int m = pr / 8, k = 2 * (pr % 8);
      *reinterpret_cast<float4*>(&L.a[buf][m * kAS + k]) = v;
    } else {
      const int k = pr / 32, m = 2 * (pr % 32);
      L.a[buf][m * kAS + k] = make_float2(v.x, v.y);
      L.a[buf][(m + 1) * kAS + k] = make_float2(v.z, v.w);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;
    const int k = pr / 32, n = 2 * (pr % 32);
    *reinterpret_cast<float4*>(&L.b[buf][k * kBS + n]) = b_val(p, st, j);
  }
}

// Lane (mi, kb) of wavefront w: rows 16w + mi.  The real K index of instruction
// (h, s) is 16h + 4kb + s (a permutation of the step's 32 real indices, applied
// identically to A and B); B column lane mi covers real column 16t + mi.
__device__ __forceinline__ void mma_f32(const LdsF32& L, int buf, int w, int lane, floatx4 (&acc)[kNT]) {
  const int mi = lane % 16, kb = lane / 16;
  const bool q = mi & 1;  // real column parity (0: Re C, 1: Im C)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float4 a = *reinterpret_cast<const float4*>(&L.a[buf][(16 * w + mi) * kAS + 8 * h + 2 * kb]);
    const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int t0 = 0; t0 < kNT; t0 += kNT / 2) {  // two halves: four independent accumulators each
      float bv[kNT / 2][4];
#pragma unroll
      for (int u = 0; u < kNT / 2; ++u) {
        const int nc = 8 * (t0 + u) + mi / 2;
        const float2 b0 = L.b[buf][(8 * h + 2 * kb) * kBS + nc];
        const float2 b1 = L.b[buf][(8 * h + 2 * kb + 1) * kBS + nc];
        // expanded B rows 2k (Re A) and 2k + 1 (Im A) at real column 2n + q
        bv[u][0] = q ? b0.y : b0.x;
        bv[u][1] = q ? b0.x : -b0.y;
        bv[u][2] = q ? b1.y : b1.x;
        bv[u][3] = q ? b1.x : -b1.y;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int u = 0; u < kNT / 2; ++u)
          acc[t0 + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[u][s], acc[t0 + u], 0, 0, 0);
    }
  }
}

// ------------------------------------------------------------------- BF16 variants
// LDS holds the operands pre-split: A as [piece][row][32 real K] and the expanded B
// as [piece][real column][32 real K], bf16, so every lane reads its 8 K values of a
// piece with one 16-byte load.
template <int NP>
struct LdsBf16 {
  __bf16 a[2][NP][kBM * kKR];
  __bf16 b[2][NP][2 * kBN * kKR];
};

template <int NP>
__device__ __forceinline__ void split(float v, __bf16 (&pc)[NP]) {
  pc[0] = (__bf16)v;
  float r = v - (float)pc[0];
  pc[1] = (__bf16)r;
  if constexpr (NP == 3) {
    r -= (float)pc[1];
    pc[2] = (__bf16)r;
  }
}

// Splits two consecutive real values and writes each piece as one bf16 pair.
template <int NP>
__device__ __forceinline__ void put2(__bf16* base, int stride_piece, float v0, float v1) {
  __bf16 p0[NP], p1[NP];
  split<NP>(v0, p0);
  split<NP>(v1, p1);
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    bf16x2 w;
    w[0] = p0[u];
    w[1] = p1[u];
    *reinterpret_cast<bf16x2*>(base + u * stride_piece) = w;
  }
}

template <int NP>
__device__ __forceinline__ void store_bf16(const CGemm& p, const Stage& st, LdsBf16<NP>& L, int buf, int tid) {
  constexpr int sa = kBM * kKR, sb = 2 * kBN * kKR;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;
    const float4 v = a_val(p, st, j);
    if (p.lda_k == 1) {  // row m, real K 4(pr % 8) .. + 3
      const int m = pr / 8, kr = 4 * (pr % 8);
      __bf16* dst = &L.a[buf][0][m * kKR + kr];
      put2<NP>(dst, sa, v.x, v.y);
      put2<NP>(dst + 2, sa, v.z, v.w);
    } else {  // rows m, m + 1, real K 2k, 2k + 1
      const int k = pr / 32, m = 2 * (pr % 32);
      put2<NP>(&L.a[buf][0][m * kKR + 2 * k], sa, v.x, v.y);
      put2<NP>(&L.a[buf][0][(m + 1) * kKR + 2 * k], sa, v.z, v.w);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int pr = tid + kMT * j;
    const int k = pr / 32, n = 2 * (pr % 32);
    const float4 v = b_val(p, st, j);
    // complex b at column n': real column 2n' holds (Re b, -Im b) at real K (2k, 2k+1),
    // real column 2n' + 1 holds (Im b, Re b)
    put2<NP>(&L.b[buf][0][(2 * n) * kKR + 2 * k], sb, v.x, -v.y);
    put2<NP>(&L.b[buf][0][(2 * n + 1) * kKR + 2 * k], sb, v.y, v.x);
    put2<NP>(&L.b[buf][0][(2 * n + 2) * kKR + 2 * k], sb, v.z, -v.w);
    put2<NP>(&L.b[buf][0][(2 * n + 3) * kKR + 2 * k], sb, v.w, v.z);
  }
}

template <int NP>
__device__ __forceinline__ void mma_bf16(const LdsBf16<NP>& L, int buf, int w, int lane, floatx4 (&acc)[kNT]) {
  const int mi = lane % 16, kb = lane / 16;
  bf16x8 ap[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) ap[u] = *reinterpret_cast<const bf16x8*>(&L.a[buf][u][(16 * w + mi) * kKR + 8 * kb]);
#pragma unroll
  for (int t = 0; t < kNT; t += 2) {
    bf16x8 b0[NP], b1[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      b0[u] = *reinterpret_cast<const bf16x8*>(&L.b[buf][u][(16 * t + mi) * kKR + 8 * kb]);
      b1[u] = *reinterpret_cast<const bf16x8*>(&L.b[buf][u][(16 * (t + 1) + mi) * kKR + 8 * kb]);
    }
    // smallest terms first; two independent accumulators interleaved
    if constexpr (NP == 3) {
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[2], b0[0], acc[t], 0, 0, 0);
      acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[2], b1[0], acc[t + 1], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], b0[1], acc[t], 0, 0, 0);
      acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], b1[1], acc[t + 1], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], b0[2], acc[t], 0, 0, 0);
      acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], b1[2], acc[t + 1], 0, 0, 0);
    }
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], b0[0], acc[t], 0, 0, 0);
    acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], b1[0], acc[t + 1], 0, 0, 0);
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], b0[1], acc[t], 0, 0, 0);
    acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], b1[1], acc[t + 1], 0, 0, 0);
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], b0[0], acc[t], 0, 0, 0);
    acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], b1[0], acc[t + 1], 0, 0, 0);
  }
}

// ------------------------------------------------------------------- epilogue
// Lane (ni, g) holds real rows 4g + i (i = 0..3) of real column 16t + ni.  Lanes ni
// and ni ^ 1 hold the real and imaginary parts of one complex column: after one
// exchange the even lane owns rows 4g, 4g + 1 and the odd lane rows 4g + 2, 4g + 3 as
// complex values.
__device__ __forceinline__ void epilogue(const CGemm& p, float2* Cp, int m0, int n0, int w, int lane,
                                         const floatx4 (&acc)[kNT]) {
  const int ni = lane % 16, g = lane / 16;
  const bool odd = ni & 1;
  const bool conj_out = p.flags & kConjC, atomic = p.flags & kAtomicC;
#pragma unroll
  for (int t = 0; t < kNT; ++t) {
    const float s0 = odd ? acc[t][0] : acc[t][2];
    const float s1 = odd ? acc[t][1] : acc[t][3];
    const float r0 = __shfl_xor(s0, 1);
    const float r1 = __shfl_xor(s1, 1);
    // even lane: (acc0, r0), (acc1, r1) for rows 4g, 4g + 1; odd: (r0, acc2), (r1, acc3)
    float2 c0 = odd ? make_float2(r0, acc[t][2]) : make_float2(acc[t][0], r0);
    float2 c1 = odd ? make_float2(r1, acc[t][3]) : make_float2(acc[t][1], r1);
    if (conj_out) {
      c0.y = -c0.y;
      c1.y = -c1.y;
    }
    const int n = n0 + 8 * t + ni / 2;
    if (n >= p.N) continue;
    const int64_t coff = p.c + col_off(n, p.c_ni, p.c_shi);
    const int mb = m0 + 16 * w + 4 * g + (odd ? 2 : 0);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = mb + i;
      if (m >= p.M) continue;
      float2* dst = Cp + coff + (int64_t)m * p.ldc_m;
      const float2 c = i ? c1 : c0;
      if (atomic) {
        atomicAdd(&dst->x, c.x);
        atomicAdd(&dst->y, c.y);
      } else {
        *dst = c;
      }
    }
  }
}

// ------------------------------------------------------------------- kernel

template <int VARIANT>
struct LdsOf {
  using type = LdsBf16<VARIANT + 1>;
};
template <>
struct LdsOf<0> {
  using type = LdsF32;
};

template <int VARIANT>
__device__ __forceinline__ void store_stage(const CGemm& p, const Stage& st, typename LdsOf<VARIANT>::type& L, int buf,
                                            int tid) {
  if constexpr (VARIANT == 0)
    store_f32(p, st, L, buf, tid);
  else
    store_bf16<VARIANT + 1>(p, st, L, buf, tid);
}

template <int VARIANT, bool AVEC>
__device__ __forceinline__ void run_tile(const CGemm& p, const CTile& tl, const float2* A, const float2* B, float2* Cp,
                                         typename LdsOf<VARIANT>::type& L) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nsteps = (p.K + kKC - 1) / kKC;
  const int nblk = (tl.n1 - tl.n0 + kBN - 1) / kBN;
  const int total = nblk * nsteps;

  floatx4 acc[kNT];
#pragma unroll
  for (int t = 0; t < kNT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  Stage st;
  load_stage<AVEC>(p, A, B, tl.m0, tl.n0, 0, tid, st);
  store_stage<VARIANT>(p, st, L, 0, tid);
  __syncthreads();
  for (int it = 0; it < total; ++it) {
    const int cur = it & 1;
    const int blk = it / nsteps, s = it - blk * nsteps;
    if (it + 1 < total) {
      const int nb = (it + 1) / nsteps, ns = (it + 1) - nb * nsteps;
      load_stage<AVEC>(p, A, B, tl.m0, tl.n0 + nb * kBN, ns * kKC, tid, st);
    }
    if constexpr (VARIANT == 0)
      mma_f32(L, cur, w, lane, acc);
    else
      mma_bf16<VARIANT + 1>(L, cur, w, lane, acc);
    if (s == nsteps - 1) {
      epilogue(p, Cp, tl.m0, tl.n0 + blk * kBN, w, lane, acc);
#pragma unroll
      for (int t = 0; t < kNT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    if (it + 1 < total) store_stage<VARIANT>(p, st, L, cur ^ 1, tid);
    __syncthreads();
  }
}

template <int VARIANT>
__global__ __launch_bounds__(kMT) void cgemm_kernel(const CGemm* __restrict__ probs, const CTile* __restrict__ tiles,
                                                    CGemmBases bases) {
  using Lds = typename LdsOf<VARIANT>::type;
  __shared__ __align__(16) Lds L;
  const CTile tl = tiles[blockIdx.x];
  const CGemm p = probs[tl.prob];
  const float2* A = base_ptr(bases, p.abase);
  const float2* B = base_ptr(bases, p.bbase);
  float2* Cp = base_ptr(bases, p.cbase);
  // 16-byte A loads need an even complex offset for every pair
  if (!((p.a | (p.lda_k == 1 ? p.lda_m : p.lda_k)) & 1))
    run_tile<VARIANT, true>(p, tl, A, B, Cp, L);
  else
    run_tile<VARIANT, false>(p, tl, A, B, Cp, L);
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
