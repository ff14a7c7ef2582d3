// Descriptors shared by the host runtime and the HIP kernels.
#pragma once
#include <cstdint>

namespace tuckfmm {

// One Tucker-compressed tensor (one group, one polarisation) inside a device arena.
// Offsets count complex elements from the start of the factor area.  Device layouts
// (chosen for coalesced streaming; the ABI uses the paper's shapes instead):
//   ubt  : U^beta transposed, [r_beta][ld_ub]          (row b = column b of U^beta)
//   core : [r_beta][ld_c], column q = theta' * r_phi + phi'
//   ut   : U^theta [n_theta][r_theta]
//   up   : U^phi [n_phi][r_phi]
//   upt  : U^phi transposed, [r_phi][n_phi]
// Row padding elements are zero.  An item with identity angular factors (the
// truncated-SVD method: r_theta = n_theta, r_phi = n_phi, U^theta = U^phi = I) has
// ident = 1, stores no angular factors, and its core is W (column q = direction).
struct alignas(16) TuckItem {
  int64_t off_ubt;
  int64_t off_core;
  int64_t off_ut;
  int64_t off_up;
  int64_t off_upt;
  int64_t row0;      // first basis row of the group
  int32_t nb, rt, rp, rb;
  int32_t ld_ub, ld_c;
  int32_t group, alpha;
  int32_t theta_first;  // 1: contract U^theta before U^phi in the angular stages
  int32_t ident;        // 1: identity angular factors (no angular products)
  int32_t frow;         // row of the item's fibre in F and G: 2 group + alpha, or alpha K + box on a box grid
  int32_t pad2;
};
static_assert(sizeof(TuckItem) == 96, "TuckItem layout");

// Work unit of the streaming kernels: a whole item (split < 0), or rows [b0, b1) of
// the item's U^beta^T and core when the item is split over several workgroups; then
// the unit writes partial sums to block `sub` of split entry `split`.
struct TuckUnit {
  int32_t item;
  int32_t b0, b1;
  int32_t split, sub;
  int32_t pad;
};
static_assert(sizeof(TuckUnit) == 24, "TuckUnit layout");

// A split item: its n_parts partial blocks, per right-hand side at
//   agg: part + r part_stride + agg_off + s q_pad   (q_pad complex values each)
//   dis: part + r part_stride + dis_off + s nb_pad  (nb_pad complex values each)
// are summed in order s = 0, 1, ... by the finishing kernel.
struct TuckSplit {
  int64_t agg_off, dis_off;
  int32_t item, n_parts;
  int32_t q_pad, nb_pad;
};
static_assert(sizeof(TuckSplit) == 32, "TuckSplit layout");

// Maxima over all items of a precision slot; they size the kernels' LDS.
struct TuckMax {
  int32_t nb, rt, rp, rb, q;
  int32_t t3;      // max of n_theta*r_phi or r_theta*n_phi intermediate
  int32_t nt, np;  // the direction grid n_theta x n_phi
  int32_t stage;   // 1: the angular products read their factors (and G) from LDS
};

// Device pointers and sizes of one uploaded precision.
//   units     : the work units (whole items and row blocks of split items)
//   order     : the units, largest first
//   pass_list : 2 n_units entries of a whole pass, largest first; entry e >= 0 is the
//               aggregation of unit e, e < 0 the disaggregation of unit ~e
//   splits    : the split items, summed by the finishing kernel
//   zero_rows : on a box grid, the rows alpha K + box of the empty boxes, which the
//               aggregation writes zero
struct TuckPlan {
  const void* factors = nullptr;
  const TuckItem* items = nullptr;
  const int32_t* order = nullptr;
  const int32_t* pass_list = nullptr;
  const int32_t* zero_rows = nullptr;  // rows of F on empty boxes (box grid only)
  int n_zero_rows = 0;
  const TuckUnit* units = nullptr;
  const TuckSplit* splits = nullptr;
  int n_units = 0, n_splits = 0;
  int64_t part_stride = 0;  // partial-sum elements per right-hand side
  void* part = nullptr;     // library-owned partial sums (device), set per call
  int32_t* next = nullptr;  // work counter of the pass kernel (device), set per call
  int n_items = 0;
  int64_t n_basis = 0;
  TuckMax mx{};
};

// One complex product C(m, n) (+)= sum_k opA(m, k) opB(k, n) of the multi-RHS path.
// Offsets and strides count complex elements from the base pointer selected by
// abase / bbase / cbase (an index into CGemmBases):
//   A(m, k) at a + m lda_m + k lda_k
//   B(k, n) at b + k ldb_k + (n / b_ni) b_shi + n % b_ni
//   C(m, n) at c + m ldc_m + (n / c_ni) c_shi + n % c_ni
enum : int32_t { kConjA = 1, kConjB = 2, kConjC = 4, kAtomicC = 8 };
struct CGemm {
  int64_t a, b, c;
  int32_t abase, bbase, cbase;
  int32_t M, N, K;
  int32_t lda_m, lda_k;
  int32_t ldb_k, b_ni, b_shi;
  int32_t ldc_m, c_ni, c_shi;
  int32_t flags;
  int32_t pad;
};
static_assert(sizeof(CGemm) == 88, "CGemm layout");

// Base pointers of a grouped launch: factors, scratch, x, F, G, V.
enum : int32_t { kBaseFactors = 0, kBaseScratch = 1, kBaseX = 2, kBaseF = 3, kBaseG = 4, kBaseV = 5 };
struct CGemmBases {
  void* p[6];
};

// One workgroup of the grouped product: rows m0 .. m0 + 63 and complex columns
// n0 .. n1 - 1 (in blocks of 32) of problem `prob`.
struct CTile {
  int32_t prob, m0, n0, n1;
};

// Dense plan: one group's rows.
struct DenseGroup {
  int64_t row0;
  int32_t nb;
  int32_t pad;
};

// Dense plan: up to kDenseBlockRows consecutive rows of one group (the work unit of
// the multi-RHS disaggregation).
constexpr int kDenseBlockRows = 16;
struct DenseBlock {
  int64_t row0;
  int32_t rows;
  int32_t group;
};

}  // namespace tuckfmm
