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
// A complex product C = A B runs on real MFMA instructions through the 2 x 2 real
// expansion of one operand: no arithmetic is wasted (8 real flops per complex
// multiply-add).  The FP32 and FP64 variants expand B,
//   [Re C, Im C] = [Re A, Im A] [[Re B, Im B], [-Im B, Re B]],
// with A read as a real matrix whose columns interleave (Re, Im) -- the stored
// layout -- and B expanded when a step is written to LDS; the bf16 variants expand A
// in registers (see their section).
//
// Workgroup tile: 64 rows x 64 complex columns, K in steps of 16 complex values (32
// real).  Four wavefronts, each owning 16 rows of the tile and eight 16 x 16 MFMA
// accumulators, of which a product of N < 64 columns runs only those its columns
// fill.  A workgroup walks its column blocks and K steps as one flat pipeline: the
// global loads of step s + 1 are in flight while step s runs on the matrix cores from
// LDS (single buffered).
//
// Arithmetic variants (factors, vectors and intermediates are complex64 in all three):
//   0  FP32    v_mfma_f32_16x16x4_f32;
//   1  BF16x2  v_mfma_f32_16x16x32_bf16; both operands are split into bf16 pieces
//              v = hi + lo on chip and each product accumulates hi*hi + hi*lo + lo*hi
//              in FP32 (the dropped lo*lo term is below 2^-16 relative);
//   2  BF16x3  three pieces v = hi + mid + lo and the six products whose order is at
//              most 2^-16 (hi*hi, hi*mid, mid*hi, hi*lo, mid*mid, lo*hi): FP32-level
//              accuracy at six bf16 instructions per product.
// Variant 3 is the complex128 path: factors, vectors and intermediates in FP64 and
// v_mfma_f64_16x16x4_f64 on them, with the same tile, pipeline and B expansion.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.hpp"
#include "kernels.hpp"

namespace tuckfmm {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMT = 256;           // threads
constexpr int kBM = 64;            // rows per tile
constexpr int kBN = 64;            // complex columns per block
constexpr int kKC = 16;            // complex K per step
constexpr int kNT = 2 * kBN / 16;  // 16-column accumulators per wavefront (8)
// FP32 A LDS row stride (complex): padding keeps 16-byte alignment and spreads banks
constexpr int kAS = kKC + 2;

__device__ __forceinline__ int64_t col_off(int n, int ni, int shi) { return (int64_t)(n / ni) * shi + n % ni; }

template <typename C2>
__device__ __forceinline__ C2* base_ptr(const CGemmBases& b, int i) {
  // i is uniform across the workgroup: a select chain, no indexed private array
  void* p = i == 0 ? b.p[0] : i == 1 ? b.p[1] : i == 2 ? b.p[2] : i == 3 ? b.p[3] : i == 4 ? b.p[4] : b.p[5];
  return static_cast<C2*>(p);
}

// ------------------------------------------------------------------ global loads
// Thread t owns four consecutive complex K values of one A row and of one B column:
//   A  K-contiguous: row t / 4, K quad t % 4;   M-contiguous: row t % 64, K quad t / 64
//   B  column t % 64, K quad t / 64
// so that a step's piece of an operand is written to LDS as whole 16-byte chunks.
// Each thread keeps a pointer to its quad that advances by one step per K step; a
// row beyond M or a column beyond N reads the operand's first elements instead.  In
// the step that holds the K tail, every element outside the product (row beyond M,
// column beyond N, K beyond the tail) is read from such a clamp address and zeroed
// when the step is written to LDS; the steps before it mask nothing (see load_stage).
// Nothing consumes the loaded values before that point, so the loads stay in flight
// while the previous step runs on the matrix cores.
template <typename C2>
struct Stage {
  C2 a[4];
  C2 b[4];
  int na, nb;  // number of valid elements (a prefix of the quad)
};

// Per-thread operand walkers.
template <typename C2>
struct Walk {
  const C2* clampa;  // first element of A
  const C2* a0;      // the thread's quad at K step 0 (clampa if the row is invalid)
  const C2* a;       // the quad at the current K step
  int64_t astep;         // pointer advance per K step (0 for an invalid row)
  int aes;               // element stride inside the quad
  int aq;                // K quad index (0..3)
  bool arow;             // row valid
  const C2* clampb;
  const C2* b;
  int64_t bstep;
  int bes;
  int bq;
  bool bcol;
};

template <typename C2>
__device__ __forceinline__ void walk_init(const CGemm& p, const C2* A, const C2* B, int m0, int tid, Walk<C2>& w) {
  const bool kc = p.lda_k == 1;
  const int am = m0 + (kc ? tid / 4 : tid % 64);
  w.aq = kc ? tid % 4 : tid / 64;
  w.arow = am < p.M;
  w.clampa = A + p.a;
  w.aes = kc ? 1 : p.lda_k;
  w.a0 = w.arow ? w.clampa + (kc ? (int64_t)am * p.lda_m + 4 * w.aq : am + (int64_t)(4 * w.aq) * p.lda_k) : w.clampa;
  w.a = w.a0;
  w.astep = w.arow ? (kc ? (int64_t)kKC : (int64_t)kKC * p.lda_k) : 0;
  w.clampb = B + p.b;
  w.bq = tid / 64;
  w.bes = p.ldb_k;
}

// Points the B walker at column block n0 (K step 0).
template <typename C2>
__device__ __forceinline__ void walk_block(const CGemm& p, int n0, int tid, Walk<C2>& w) {
  const int n = n0 + tid % 64;
  w.bcol = n < p.N;
  w.b = w.bcol ? w.clampb + col_off(n, p.b_ni, p.b_shi) + (int64_t)(4 * w.bq) * p.ldb_k : w.clampb;
  w.bstep = w.bcol ? (int64_t)kKC * p.ldb_k : 0;
  w.a = w.a0;
}

// AVEC (uniform per product; K-contiguous A with even offset and row stride): A is
// read as two 16-byte pairs.  A pair whose first element is valid is read whole; at
// an odd K its second element is the row's zero padding (factor rows are padded to
// an even length) and is masked.  (A complex128 element is a 16-byte load by itself.)
// FULL (uniform): the step lies inside K (k0 + 16 <= K).  Then no element is masked:
// a row beyond M or a column beyond N reads the operand's first elements (valid, as
// K >= 16) and only feeds accumulator rows or columns that the epilogue never stores,
// so the step needs no per-element selects.  Only the step holding the K tail masks.
template <bool AVEC, bool FULL, typename C2>
__device__ __forceinline__ void load_stage(const CGemm& p, int k0, Walk<C2>& w, Stage<C2>& st) {
  int na = 4, nb = 4;
  if constexpr (!FULL) {
    na = w.arow ? min(4, max(0, p.K - k0 - 4 * w.aq)) : 0;
    nb = w.bcol ? min(4, max(0, p.K - k0 - 4 * w.bq)) : 0;
  }
  const C2* pa = FULL || na > 0 ? w.a : w.clampa;
  if constexpr (AVEC) {
    static_assert(sizeof(C2) == 8, "paired loads are for complex64");
    const float4 u = *reinterpret_cast<const float4*>(pa);
    const float4 v = *reinterpret_cast<const float4*>(pa + (FULL || na > 2 ? 2 : 0));
    st.a[0] = make_float2(u.x, u.y);
    st.a[1] = make_float2(u.z, u.w);
    st.a[2] = make_float2(v.x, v.y);
    st.a[3] = make_float2(v.z, v.w);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) st.a[e] = pa[FULL || e < na ? e * w.aes : 0];
  }
  const C2* pb = FULL || nb > 0 ? w.b : w.clampb;
#pragma unroll
  for (int e = 0; e < 4; ++e) st.b[e] = pb[FULL || e < nb ? e * w.bes : 0];
  st.na = na;
  st.nb = nb;
  w.a += w.astep;
  w.b += w.bstep;
}

// Conjugation flips the sign bit of the imaginary part: conj is 0 or 0x80000000,
// uniform per product (one XOR, no select).
__device__ __forceinline__ float flip_sign(float v, uint32_t conj) { return __uint_as_float(__float_as_uint(v) ^ conj); }
__device__ __forceinline__ double flip_sign(double v, uint32_t conj) {
  return __longlong_as_double(__double_as_longlong(v) ^ (long long)((uint64_t)conj << 32));
}

__device__ __forceinline__ uint32_t conj_mask(const CGemm& p, int flag) { return (p.flags & flag) ? 0x80000000u : 0u; }

// Element e of the stage's A (B) values with invalid elements zeroed (not in a FULL
// step) and the conjugation applied -- the point where the loads are waited for.
template <bool FULL, typename C2>
__device__ __forceinline__ C2 a_val(const Stage<C2>& st, int e, uint32_t conj) {
  C2 v = FULL || e < st.na ? st.a[e] : czero<C2>();
  v.y = flip_sign(v.y, conj);
  return v;
}

template <bool FULL, typename C2>
__device__ __forceinline__ C2 b_val(const Stage<C2>& st, int e, uint32_t conj) {
  C2 v = FULL || e < st.nb ? st.b[e] : czero<C2>();
  v.y = flip_sign(v.y, conj);
  return v;
}

// Row / K quad of the thread's A values in the tile (see walk_init).
__device__ __forceinline__ void a_slot(const CGemm& p, int tid, int& m, int& kq) {
  if (p.lda_k == 1) {
    m = tid / 4;
    kq = tid % 4;
  } else {
    m = tid % 64;
    kq = tid / 64;
  }
}

// ------------------------------------------------------------------- FP32 variant
// LDS: A complex [row][K]; B already expanded, [K][complex column][q] with q = 0 the
// pair (Re b, -Im b) and q = 1 the pair (Im b, Re b): the expanded-B values a lane
// with column parity q needs for real rows 2k and 2k + 1.
constexpr int kXS = 2 * kBN + 4;  // expanded-B row stride (float2)

struct LdsF32 {
  float2 a[kBM * kAS];
  float2 b[kKC * kXS];
};

template <bool FULL>
__device__ __forceinline__ void store_f32(const CGemm& p, const Stage<float2>& st, LdsF32& L, int tid, uint32_t ca,
                                          uint32_t cb) {
  int m, kq;
  a_slot(p, tid, m, kq);
  float2* da = &L.a[m * kAS + 4 * kq];
  const float2 a0 = a_val<FULL>(st, 0, ca), a1 = a_val<FULL>(st, 1, ca), a2 = a_val<FULL>(st, 2, ca),
               a3 = a_val<FULL>(st, 3, ca);
  *reinterpret_cast<float4*>(da) = make_float4(a0.x, a0.y, a1.x, a1.y);
  *reinterpret_cast<float4*>(da + 2) = make_float4(a2.x, a2.y, a3.x, a3.y);
  const int nn = tid % 64, kb = 4 * (tid / 64);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float2 v = b_val<FULL>(st, e, cb);
    *reinterpret_cast<float4*>(&L.b[(kb + e) * kXS + 2 * nn]) = make_float4(v.x, -v.y, v.y, v.x);
  }
}

// Lane (mi, kb) of wavefront w: rows 16w + mi.  The real K index of instruction
// (h, s) is 16h + 4kb + s (a permutation of the step's 32 real indices, applied
// identically to A and B); B column lane mi covers real column 16t + mi.  Only the
// NTE accumulators (16 real columns each) that hold columns of the product run: a
// product of N complex columns needs ceil(N / 8).  (The MFMA sequence is
// straight-line code: a branch around it would make the compiler move the
// accumulators between register files.)
template <int NTE>
__device__ __forceinline__ void mma_f32(const LdsF32& L, int w, int lane, floatx4 (&acc)[NTE]) {
  const int mi = lane % 16, kb = lane / 16;
  constexpr int kG = NTE < 4 ? NTE : 4;  // accumulators per group of independent MFMAs
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float4 a = *reinterpret_cast<const float4*>(&L.a[(16 * w + mi) * kAS + 8 * h + 2 * kb]);
    const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int t0 = 0; t0 < NTE; t0 += kG) {
      float2 b0[kG], b1[kG];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int col = 16 * (t0 + u) + mi;  // = 2 (complex column) + q
        b0[u] = L.b[(8 * h + 2 * kb) * kXS + col];
        b1[u] = L.b[(8 * h + 2 * kb + 1) * kXS + col];
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], b0[u].x, acc[t0 + u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], b0[u].y, acc[t0 + u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], b1[u].x, acc[t0 + u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], b1[u].y, acc[t0 + u], 0, 0, 0);
    }
  }
}

// ------------------------------------------------------------------- FP64 variant
// The FP32 layout with double2 values (52 KB of LDS).  v_mfma_f64_16x16x4_f64 takes
// its operands in the lane layout of the FP32 instruction (A row l % 16, B column
// l % 16, K index l / 16), so the real K permutation and the B reads are those of
// mma_f32; only the accumulator layout differs (see the epilogue).
struct LdsF64 {
  double2 a[kBM * kAS];
  double2 b[kKC * kXS];
};

template <bool FULL>
__device__ __forceinline__ void store_f64(const CGemm& p, const Stage<double2>& st, LdsF64& L, int tid, uint32_t ca,
                                          uint32_t cb) {
  int m, kq;
  a_slot(p, tid, m, kq);
  double2* da = &L.a[m * kAS + 4 * kq];
#pragma unroll
  for (int e = 0; e < 4; ++e) da[e] = a_val<FULL>(st, e, ca);
  const int nn = tid % 64, kb = 4 * (tid / 64);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double2 v = b_val<FULL>(st, e, cb);
    double2* db = &L.b[(kb + e) * kXS + 2 * nn];
    db[0] = make_double2(v.x, -v.y);
    db[1] = make_double2(v.y, v.x);
  }
}

template <int NTE>
__device__ __forceinline__ void mma_f64(const LdsF64& L, int w, int lane, doublex4 (&acc)[NTE]) {
  const int mi = lane % 16, kb = lane / 16;
  constexpr int kG = NTE < 4 ? NTE : 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double2* pa = &L.a[(16 * w + mi) * kAS + 8 * h + 2 * kb];
    const double2 a0 = pa[0], a1 = pa[1];
    const double av[4] = {a0.x, a0.y, a1.x, a1.y};
#pragma unroll
    for (int t0 = 0; t0 < NTE; t0 += kG) {
      double2 b0[kG], b1[kG];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int col = 16 * (t0 + u) + mi;
        b0[u] = L.b[(8 * h + 2 * kb) * kXS + col];
        b1[u] = L.b[(8 * h + 2 * kb + 1) * kXS + col];
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], b0[u].x, acc[t0 + u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], b0[u].y, acc[t0 + u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[2], b1[u].x, acc[t0 + u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < kG; ++u) acc[t0 + u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[3], b1[u].y, acc[t0 + u], 0, 0, 0);
    }
  }
}

// ------------------------------------------------------------------- BF16 variants
// Complex products on bf16 MFMA with the 2 x 2 real expansion on the A side:
//   real row 2m     (Re a, -Im a) per complex K value    gives  Re c
//   real row 2m + 1 (Im a,  Re a)                          gives  Im c
// against B as stored, (Re b, Im b) per complex K value.  Operands are staged in LDS
// as words holding one complex value's bf16 piece (Re | Im << 16): B words feed the
// MFMA unchanged, and the words of real A row 2m + q are the staged word with its high
// half negated (q = 0) or its halves swapped (q = 1), formed in registers after the LDS
// read; the two lanes of a complex row read the same LDS address.  Compared with
// expanding B, LDS holds half the B bytes and a wavefront reads 6 instead of 9 16-byte
// fragments per piece and K step.  The factors and intermediates are complex64 in HBM
// and are split when a step is written to LDS.
// LDS per piece: A [64 complex rows][16 words], B [64 complex columns][16 words], rows
// padded to 20 words.  Wavefront w owns complex rows 16w .. 16w + 15 (two MFMA blocks
// of 8 complex rows) and the 64 complex columns (four MFMA blocks of 16 columns), of
// which a product of N < 64 columns runs only the ceil(N / 16) blocks its columns fill
// (rounded up to 1, 2 or 4).
constexpr int kWS = kKC + 4;  // word row stride
constexpr int kNB = kBN / 16;  // 16-column blocks per tile (4)

template <int NP>
struct LdsBf16 {
  uint32_t a[NP][kBM * kWS];
  uint32_t b[NP][kBN * kWS];
};

// The NP words of a complex value v: word u holds the bf16 pieces u of Re v (low half)
// and Im v (high half), v ~ sum of the pieces, each piece the round-to-nearest bf16 of
// what the earlier pieces leave.  Both parts convert in one packed instruction, and a
// half widens back to FP32 by its position (shift or mask).
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
template <int NP>
__device__ __forceinline__ void split_words(float2 v, uint32_t (&w)[NP]) {
  floatx2 r = {v.x, v.y};
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    w[u] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
    if (u + 1 < NP) {
      r.x -= __builtin_bit_cast(float, w[u] << 16);
      r.y -= __builtin_bit_cast(float, w[u] & 0xffff0000u);
    }
  }
}

// A and B are loaded by the FP32 variant's walkers and split into bf16 pieces when the
// step is written to LDS, with the invalid elements zeroed and the conjugation flags
// applied.
template <int NP, bool FULL>
__device__ __forceinline__ void store_stage_b16(const CGemm& p, const Stage<float2>& st, LdsBf16<NP>& L, int tid,
                                                 uint32_t ca, uint32_t cb) {
  {
    int m, kq;
    a_slot(p, tid, m, kq);
    uint32_t w[NP][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t pc[NP];
      split_words<NP>(a_val<FULL>(st, e, ca), pc);
#pragma unroll
      for (int u = 0; u < NP; ++u) w[u][e] = pc[u];
    }
#pragma unroll
    for (int u = 0; u < NP; ++u)
      *reinterpret_cast<uint4*>(&L.a[u][m * kWS + 4 * kq]) = make_uint4(w[u][0], w[u][1], w[u][2], w[u][3]);
  }
  const int nn = tid % 64, kq = tid / 64;
  uint32_t w[NP][4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t pc[NP];
    split_words<NP>(b_val<FULL>(st, e, cb), pc);
#pragma unroll
    for (int u = 0; u < NP; ++u) w[u][e] = pc[u];
  }
#pragma unroll
  for (int u = 0; u < NP; ++u)
    *reinterpret_cast<uint4*>(&L.b[u][nn * kWS + 4 * kq]) = make_uint4(w[u][0], w[u][1], w[u][2], w[u][3]);
}

template <int NP>
__device__ __forceinline__ void mma_pair(const bf16x8 (&ap)[NP], const bf16x8 (&bp)[NP], floatx4& acc) {
  // smallest terms first
  if constexpr (NP == 3) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[2], bp[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], bp[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], bp[2], acc, 0, 0, 0);
  }
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[1], bp[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], bp[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[0], bp[0], acc, 0, 0, 0);
}

// Lane (mi, kb) of wavefront w: real A row mi of each 16-row block (complex row
// 16w + 8rb + mi / 2, part mi & 1), B column 16t + mi, complex K values 4kb .. 4kb + 3
// (real K 8kb .. 8kb + 7, the same order in A and B).
template <int NP, int NTB>
__device__ __forceinline__ void mma_bf16(const LdsBf16<NP>& L, int w, int lane, floatx4 (&acc)[2][NTB]) {
  const int mi = lane % 16, kb = lane / 16;
  const uint32_t rot = (mi & 1) ? 16u : 0u;            // swap the halves: (Im a, Re a)
  const uint32_t flip = (mi & 1) ? 0u : 0x80000000u;   // negate the high half: (Re a, -Im a)
  bf16x8 ap[2][NP];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      uint4 v = *reinterpret_cast<const uint4*>(&L.a[u][(16 * w + 8 * rb + mi / 2) * kWS + 4 * kb]);
      v.x = __builtin_rotateright32(v.x, rot) ^ flip;
      v.y = __builtin_rotateright32(v.y, rot) ^ flip;
      v.z = __builtin_rotateright32(v.z, rot) ^ flip;
      v.w = __builtin_rotateright32(v.w, rot) ^ flip;
      ap[rb][u] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
  for (int t = 0; t < NTB; ++t) {
    bf16x8 bp[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u)
      bp[u] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&L.b[u][(16 * t + mi) * kWS + 4 * kb]));
    mma_pair<NP>(ap[0], bp, acc[0][t]);
    mma_pair<NP>(ap[1], bp, acc[1][t]);
  }
}

// Accumulator register i of lane (ni, g) in block (rb, t) holds real row 4g + i of the
// block: complex row 16w + 8rb + 2g + i / 2, real part for even i, imaginary for odd,
// of complex column 16t + ni.  Every lane thus holds whole complex values.
template <int NTB>
__device__ __forceinline__ void epilogue_b16(const CGemm& p, float2* Cp, int m0, int n0, int w, int lane,
                                             const floatx4 (&acc)[2][NTB]) {
  const int ni = lane % 16, g = lane / 16;
  const bool conj_out = p.flags & kConjC, atomic = p.flags & kAtomicC;
#pragma unroll
  for (int t = 0; t < NTB; ++t) {
    const int n = n0 + 16 * t + ni;
    if (n >= p.N) continue;
    const int64_t coff = p.c + col_off(n, p.c_ni, p.c_shi);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int m = m0 + 16 * w + 8 * rb + 2 * g + i;
        if (m >= p.M) continue;
        float2 c = make_float2(acc[rb][t][2 * i], acc[rb][t][2 * i + 1]);
        if (conj_out) c.y = -c.y;
        float2* dst = Cp + coff + (int64_t)m * p.ldc_m;
        if (atomic) {
          atomicAdd(&dst->x, c.x);
          atomicAdd(&dst->y, c.y);
        } else {
          *dst = c;
        }
      }
  }
}

// ------------------------------------------------------------------- epilogue
// Accumulator register i of lane (ni, g) holds real column 16t + ni of real row
//   4g + i   (FP32 instruction),   4i + g   (FP64 instruction).
// Lanes ni and ni ^ 1 hold the real and imaginary parts of one complex column: after
// one exchange the even lane owns the rows of registers 0, 1 and the odd lane those
// of registers 2, 3 as complex values.
template <typename C2, typename ACC, int NTE>
__device__ __forceinline__ void epilogue(const CGemm& p, C2* Cp, int m0, int n0, int w, int lane,
                                         const ACC (&acc)[NTE]) {
  using R = decltype(C2{}.x);
  constexpr bool kF64 = sizeof(R) == 8;
  const int ni = lane % 16, g = lane / 16;
  const bool odd = ni & 1;
  const bool conj_out = p.flags & kConjC, atomic = p.flags & kAtomicC;
#pragma unroll
  for (int t = 0; t < NTE; ++t) {
    const R s0 = odd ? acc[t][0] : acc[t][2];
    const R s1 = odd ? acc[t][1] : acc[t][3];
    const R r0 = __shfl_xor(s0, 1);
    const R r1 = __shfl_xor(s1, 1);
    // even lane: (acc0, r0), (acc1, r1) for registers 0, 1; odd: (r0, acc2), (r1, acc3)
    C2 c0 = odd ? C2{r0, acc[t][2]} : C2{acc[t][0], r0};
    C2 c1 = odd ? C2{r1, acc[t][3]} : C2{acc[t][1], r1};
    if (conj_out) {
      c0.y = -c0.y;
      c1.y = -c1.y;
    }
    const int n = n0 + 8 * t + ni / 2;
    if (n >= p.N) continue;
    const int64_t coff = p.c + col_off(n, p.c_ni, p.c_shi);
    const int reg0 = odd ? 2 : 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + 16 * w + (kF64 ? 4 * (reg0 + i) + g : 4 * g + reg0 + i);
      if (m >= p.M) continue;
      C2* dst = Cp + coff + (int64_t)m * p.ldc_m;
      const C2 c = i ? c1 : c0;
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

// Per-variant types (LDS stage, complex element, accumulator) and the wavefronts per
// SIMD the register allocation is held to.  More resident wavefronts hide more of the
// operand-load latency: FP32, BF16x2 and BF16x3 run 4, FP64 3 (its 52 KB of LDS allows
// no more).  BF16x3 and FP64 then spill 10 and 15 registers, all outside the K loop
// (where a column block starts or ends); on the 64-RHS pass of the 30-lambda sphere
// they take 6% and 5% less time than at 3 and 2.  FP32 at 5 spills 54 registers, four
// of them reloaded in every K step, and ran 9% slower; BF16x2 at 5 would spill 57.
template <int VARIANT>
struct VarOf {
  using lds = LdsBf16<VARIANT + 1>;
  using c2 = float2;
  using acc = floatx4;
  static constexpr int waves = 4;
};
template <>
struct VarOf<0> {
  using lds = LdsF32;
  using c2 = float2;
  using acc = floatx4;
  static constexpr int waves = 4;
};
template <>
struct VarOf<3> {
  using lds = LdsF64;
  using c2 = double2;
  using acc = doublex4;
  static constexpr int waves = 3;
};

template <int VARIANT, bool FULL>
__device__ __forceinline__ void store_stage(const CGemm& p, const Stage<typename VarOf<VARIANT>::c2>& st,
                                            typename VarOf<VARIANT>::lds& L, int tid, uint32_t ca, uint32_t cb) {
  if constexpr (VARIANT == 0)
    store_f32<FULL>(p, st, L, tid, ca, cb);
  else if constexpr (VARIANT == 3)
    store_f64<FULL>(p, st, L, tid, ca, cb);
  else
    store_stage_b16<VARIANT + 1, FULL>(p, st, L, tid, ca, cb);
}

// Loads one step (k0 = ns * 16) in the form its position in K allows; the same test
// picks the matching store.
template <bool AVEC, typename C2>
__device__ __forceinline__ void load_step(const CGemm& p, bool full, int ns, Walk<C2>& w, Stage<C2>& st) {
  if (full)
    load_stage<AVEC, true>(p, ns * kKC, w, st);
  else
    load_stage<AVEC, false>(p, ns * kKC, w, st);
}

template <int VARIANT>
__device__ __forceinline__ void store_step(const CGemm& p, bool full, const Stage<typename VarOf<VARIANT>::c2>& st,
                                           typename VarOf<VARIANT>::lds& L, int tid, uint32_t ca, uint32_t cb) {
  if (full)
    store_stage<VARIANT, true>(p, st, L, tid, ca, cb);
  else
    store_stage<VARIANT, false>(p, st, L, tid, ca, cb);
}

template <int VARIANT, int NTE>
__device__ __forceinline__ void mma_stage(const typename VarOf<VARIANT>::lds& L, int w, int lane,
                                          typename VarOf<VARIANT>::acc (&acc)[NTE]) {
  if constexpr (VARIANT == 0)
    mma_f32<NTE>(L, w, lane, acc);
  else if constexpr (VARIANT == 3)
    mma_f64<NTE>(L, w, lane, acc);
  else
    mma_bf16<VARIANT + 1, NTE>(L, w, lane, acc);
}

// One tile: column blocks n0 = tl.n0, tl.n0 + 64, ... below tl.n1, each a full K
// sweep, walked as one pipeline over (block, K step).  LDS is single buffered: the
// loads of the next step are issued before the current step's matrix-core work and
// written to LDS after it.  A wavefront whose 16 rows lie past the problem's M
// (ACTIVE = false: the angular products have M = r_theta, r_phi, n_theta or n_phi,
// often well below the 64-row tile) still loads, stores and meets every barrier, but
// issues no matrix-core work, leaving the matrix cores to the other wavefronts.  An
// active wavefront runs NTE of the eight 16-column accumulators: the products with
// N = rc columns (the beta and core contractions, most of the work) need only
// ceil(rc / 8) of them when fewer than 64 right-hand sides share a chunk.
template <int VARIANT, bool AVEC, bool ACTIVE, int NTE>
__device__ __forceinline__ void run_tile(const CGemm& p, const CTile& tl, const typename VarOf<VARIANT>::c2* A,
                                         const typename VarOf<VARIANT>::c2* B, typename VarOf<VARIANT>::c2* Cp,
                                         typename VarOf<VARIANT>::lds& L) {
  using C2 = typename VarOf<VARIANT>::c2;
  using ACC = typename VarOf<VARIANT>::acc;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nsteps = (p.K + kKC - 1) / kKC;

  ACC acc[NTE];
  if constexpr (ACTIVE) {
#pragma unroll
    for (int t = 0; t < NTE; ++t) acc[t] = ACC{0, 0, 0, 0};
  }
  Walk<C2> wk;
  walk_init(p, A, B, tl.m0, tid, wk);
  walk_block(p, tl.n0, tid, wk);
  const uint32_t ca = conj_mask(p, kConjA), cb = conj_mask(p, kConjB);
  Stage<C2> st;
  load_step<AVEC>(p, kKC <= p.K, 0, wk, st);
  store_step<VARIANT>(p, kKC <= p.K, st, L, tid, ca, cb);
  __syncthreads();
  for (int n0 = tl.n0;;) {
    // K sweep of one column block; the epilogue stays outside this loop so that the
    // accumulators never cross a branch inside it
    for (int s = 0; s < nsteps; ++s) {
      int nn0 = n0, ns = s + 1;
      if (ns == nsteps) {
        ns = 0;
        nn0 += kBN;
      }
      const bool more = nn0 < tl.n1, full = (ns + 1) * kKC <= p.K;
      if (more) {
        if (ns == 0) walk_block(p, nn0, tid, wk);
        load_step<AVEC>(p, full, ns, wk, st);
      }
      if constexpr (ACTIVE) mma_stage<VARIANT, NTE>(L, w, lane, acc);
      if (more) {
        __syncthreads();  // every wavefront is done reading the step
        store_step<VARIANT>(p, full, st, L, tid, ca, cb);
        __syncthreads();
      }
    }
    if constexpr (ACTIVE) epilogue(p, Cp, tl.m0, n0, w, lane, acc);
    n0 += kBN;
    if (n0 >= tl.n1) break;
    if constexpr (ACTIVE) {
#pragma unroll
      for (int t = 0; t < NTE; ++t) acc[t] = ACC{0, 0, 0, 0};
    }
  }
}

// The wavefront's rows (uniform per wavefront) and the product's width (uniform per
// workgroup) select the instantiation.
template <int VARIANT, bool AVEC>
__device__ __forceinline__ void run_tile_of(const CGemm& p, const CTile& tl, const typename VarOf<VARIANT>::c2* A,
                                            const typename VarOf<VARIANT>::c2* B, typename VarOf<VARIANT>::c2* Cp,
                                            typename VarOf<VARIANT>::lds& L) {
  if (tl.m0 + 16 * (int)(threadIdx.x >> 6) >= p.M)
    run_tile<VARIANT, AVEC, false, 1>(p, tl, A, B, Cp, L);
  else if (p.N <= 8)
    run_tile<VARIANT, AVEC, true, 1>(p, tl, A, B, Cp, L);
  else if (p.N <= 16)
    run_tile<VARIANT, AVEC, true, 2>(p, tl, A, B, Cp, L);
  else if (p.N <= 32)
    run_tile<VARIANT, AVEC, true, 4>(p, tl, A, B, Cp, L);
  else
    run_tile<VARIANT, AVEC, true, kNT>(p, tl, A, B, Cp, L);
}

// The bf16 variants: the pipeline of run_tile with the split at the LDS store.
template <int VARIANT, bool AVEC, bool ACTIVE, int NTB>
__device__ __forceinline__ void run_tile_b16(const CGemm& p, const CTile& tl, const float2* A, const float2* B,
                                              float2* Cp, typename VarOf<VARIANT>::lds& L) {
  constexpr int NP = VARIANT + 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nsteps = (p.K + kKC - 1) / kKC;

  floatx4 acc[2][NTB];
  if constexpr (ACTIVE) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int t = 0; t < NTB; ++t) acc[rb][t] = floatx4{0, 0, 0, 0};
  }
  Walk<float2> wk;
  walk_init(p, A, B, tl.m0, tid, wk);
  walk_block(p, tl.n0, tid, wk);
  const uint32_t ca = conj_mask(p, kConjA), cb = conj_mask(p, kConjB);
  Stage<float2> st;
  load_step<AVEC>(p, kKC <= p.K, 0, wk, st);
  store_step<VARIANT>(p, kKC <= p.K, st, L, tid, ca, cb);
  __syncthreads();
  for (int n0 = tl.n0;;) {
    for (int s = 0; s < nsteps; ++s) {
      int nn0 = n0, ns = s + 1;
      if (ns == nsteps) {
        ns = 0;
        nn0 += kBN;
      }
      const bool more = nn0 < tl.n1, full = (ns + 1) * kKC <= p.K;
      if (more) {
        if (ns == 0) walk_block(p, nn0, tid, wk);
        load_step<AVEC>(p, full, ns, wk, st);
      }
      if constexpr (ACTIVE) mma_bf16<NP, NTB>(L, w, lane, acc);
      if (more) {
        __syncthreads();  // every wavefront is done reading the step
        store_step<VARIANT>(p, full, st, L, tid, ca, cb);
        __syncthreads();
      }
    }
    if constexpr (ACTIVE) epilogue_b16<NTB>(p, Cp, tl.m0, n0, w, lane, acc);
    n0 += kBN;
    if (n0 >= tl.n1) break;
    if constexpr (ACTIVE) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int t = 0; t < NTB; ++t) acc[rb][t] = floatx4{0, 0, 0, 0};
    }
  }
}

template <int VARIANT, bool AVEC>
__device__ __forceinline__ void run_tile_of_b16(const CGemm& p, const CTile& tl, const float2* A, const float2* B,
                                                 float2* Cp, typename VarOf<VARIANT>::lds& L) {
  if (tl.m0 + 16 * (int)(threadIdx.x >> 6) >= p.M)
    run_tile_b16<VARIANT, AVEC, false, 1>(p, tl, A, B, Cp, L);
  else if (p.N <= 16)
    run_tile_b16<VARIANT, AVEC, true, 1>(p, tl, A, B, Cp, L);
  else if (p.N <= 32)
    run_tile_b16<VARIANT, AVEC, true, 2>(p, tl, A, B, Cp, L);
  else
    run_tile_b16<VARIANT, AVEC, true, kNB>(p, tl, A, B, Cp, L);
}

template <int VARIANT>
__global__ __launch_bounds__(kMT) __attribute__((amdgpu_waves_per_eu(VarOf<VARIANT>::waves, 8))) void cgemm_kernel(const CGemm* __restrict__ probs, const CTile* __restrict__ tiles,
                                                    CGemmBases bases) {
  using Lds = typename VarOf<VARIANT>::lds;
  using C2 = typename VarOf<VARIANT>::c2;
  __shared__ __align__(16) Lds L;
  const CTile tl = tiles[blockIdx.x];
  const CGemm p = probs[tl.prob];
  const C2* A = base_ptr<C2>(bases, p.abase);
  const C2* B = base_ptr<C2>(bases, p.bbase);
  C2* Cp = base_ptr<C2>(bases, p.cbase);
  // paired 16-byte A loads (complex64): K-contiguous A with an even offset and row
  // stride
  if constexpr (VARIANT == 1 || VARIANT == 2) {
    if (p.lda_k == 1 && !((p.a | p.lda_m) & 1))
      run_tile_of_b16<VARIANT, true>(p, tl, A, B, Cp, L);
    else
      run_tile_of_b16<VARIANT, false>(p, tl, A, B, Cp, L);
  } else if constexpr (VARIANT == 3) {
    run_tile_of<VARIANT, false>(p, tl, A, B, Cp, L);
  } else {
    if (p.lda_k == 1 && !((p.a | p.lda_m) & 1))
      run_tile_of<VARIANT, true>(p, tl, A, B, Cp, L);
    else
      run_tile_of<VARIANT, false>(p, tl, A, B, Cp, L);
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
  else if (variant == 3)
    hipLaunchKernelGGL(cgemm_kernel<3>, dim3(n_tiles), dim3(kMT), 0, s, probs, tiles, b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_zero_cplx(size_t elem_bytes, void* v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(mrhs_zero_kernel<double2>, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<double2*>(v), n);
  else
    hipLaunchKernelGGL(mrhs_zero_kernel<float2>, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<float2*>(v), n);
  return hipGetLastError();
}

}  // namespace tuckfmm
