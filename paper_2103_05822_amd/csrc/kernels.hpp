// Host-side launchers of the HIP kernels (implemented in the *.hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "desc.hpp"

namespace tuckfmm {

// Tucker aggregation / disaggregation / whole pass over an uploaded plan, one
// workgroup of `threads` (64, 128, 256 or 512) per item and right-hand side.
template <typename T>
hipError_t launch_tucker_agg(const TuckPlan& pl, int threads, int n_theta, int n_phi, int nrhs, const void* x,
                             void* F, hipStream_t s);
template <typename T>
hipError_t launch_tucker_disagg(const TuckPlan& pl, int threads, int n_theta, int n_phi, int nrhs, const void* G,
                                void* V, hipStream_t s);
template <typename T>
hipError_t launch_tucker_pass(const TuckPlan& pl, int threads, int n_theta, int n_phi, int nrhs, const void* x,
                              void* F, const void* G, void* V, hipStream_t s);
// Largest dynamic LDS request of the Tucker kernels.
template <typename T>
size_t tucker_lds_bytes(const TuckMax& mx);

// Grouped complex GEMM of the multi-RHS path (variant 0: FP32 MFMA, 1: BF16 two-piece
// split, 2: BF16 three-piece split, all on complex64 data with FP32 accumulation;
// 3: FP64 MFMA on complex128 data), one workgroup per tile.
hipError_t launch_cgemm(int variant, const CGemm* probs, const CTile* tiles, int n_tiles, const CGemmBases& b,
                        hipStream_t s);
// Zero n complex values of elem_bytes (8 or 16) each.
hipError_t launch_zero_cplx(size_t elem_bytes, void* v, int64_t n, hipStream_t s);
// Zero rows[0 .. n_rows) of a row-major array of rows of row_elems complex values of
// elem_bytes (8 or 16) each.
hipError_t launch_zero_rows(size_t elem_bytes, void* base, const int32_t* rows, int n_rows, int64_t row_elems,
                            hipStream_t s);

// Dense (plain) aggregation / disaggregation.
template <typename T>
hipError_t launch_dense_agg(const void* A, const DenseGroup* groups, int n_groups, int ncols, int nrhs,
                            const void* x, void* F, hipStream_t s);
template <typename T>
hipError_t launch_dense_disagg(const void* A, const int64_t* offsets, int n_groups, int64_t n_rows,
                               const DenseBlock* blocks, int n_blocks, int ncols, int nrhs, const void* G, void* V,
                               hipStream_t s);

// Far-field fill, eq. (4): rowdata [rows][kRowDoubles], dirs [ndir][9].
constexpr int kRowDoubles = 40;  // 6 points x (rel xyz, rho xyz) + scale + box centre
hipError_t launch_farfield_fill(const double* rowdata, int64_t rows, const double* dirs, int ndir, double k,
                                void* out, hipStream_t s);
// Plane-wave excitation of eq. (2): out [rows][nrhs] complex (elem_bytes 8 or 16),
// waves [nrhs][6] = (k_hat, e_hat) on the device.
hipError_t launch_planewave(const double* rowdata, int64_t rows, const double* waves, int nrhs, double k,
                            size_t elem_bytes, void* out, hipStream_t s);

// Precision conversion / packing helpers for setup.
// Gram matrices of the theta and phi unfoldings of a slab [nb][nt][np] (column-major
// outputs); `part` holds mode_gram_chunks(nb) * (nt*nt + np*np) complex values.
constexpr int kGramRows = 8;
int mode_gram_chunks(int nb);
hipError_t launch_mode_gram(const void* slab, int nb, int nt, int np, void* part, void* gt, void* gp,
                            hipStream_t s);
hipError_t launch_select_cols_rev(const void* src, int n, int r, void* dst, hipStream_t s);
// out[k] = sum_l |a[k sk + l sl]|^2, k < K, l < L (complex128 a, FP64 sums).
hipError_t launch_strided_energy(const void* a, int K, int64_t sk, int64_t L, int64_t sl, double* out,
                                 hipStream_t s);
hipError_t launch_gather_slab(const void* farfield, int64_t row0, int nb, int alpha, int n_theta, int n_phi,
                              void* out_tp, void* out_pt, hipStream_t s);

}  // namespace tuckfmm
