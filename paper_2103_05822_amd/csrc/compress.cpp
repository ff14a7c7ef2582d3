// Setup: truncated HOSVD of the dense far-field tensors (Section II.B, eq. (6)),
// FP64 on the device.
//
// For each (group, polarisation) tensor A (n_theta x n_phi x n_beta):
//   1. the three mode unfoldings' Gram matrices with rocBLAS ZHERK;
//   2. their Hermitian eigendecompositions with rocSOLVER ZHEEVD: the eigenvectors
//      are the left singular vectors of the unfoldings and the eigenvalues their
//      squared singular values;
//   3. per mode, the smallest rank whose discarded tail satisfies
//      sum_{i>=r} s_i^2 <= gamma^2/3 ||A||_F^2 (host, FP64);
//   4. the core C = A x_3 U^beta* x_1 U^theta* x_2 U^phi* with three ZGEMMs.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "kernels.hpp"

using namespace tuckfmm;

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct BlasHandle {
  rocblas_handle h = nullptr;
  ~BlasHandle() {
    if (h) rocblas_destroy_handle(h);
  }
};

#define TFMM_BLAS(expr)                                                                \
  do {                                                                                 \
    rocblas_status s_ = (expr);                                                        \
    if (s_ != rocblas_status_success)                                                  \
      return fail(FMM_ERR_DEVICE, "%s failed: %s", #expr, rocblas_status_to_string(s_)); \
  } while (0)

// Smallest r >= 1 with sum_{i >= r} lam_desc[i] <= thr2 (lam sorted descending);
// thr2 <= 0 keeps everything.
int truncation_rank(const std::vector<double>& lam_desc, double thr2) {
  const int n = (int)lam_desc.size();
  if (thr2 <= 0.0) return n;
  double tail = 0.0;
  int r = n;
  // walk from the smallest eigenvalue up while the tail stays within the budget
  for (int i = n - 1; i >= 1; --i) {
    tail += std::max(lam_desc[i], 0.0);
    if (tail <= thr2) r = i;
    else break;
  }
  return std::max(r, 1);
}

}  // namespace

extern "C" fmm_status fmm_farfield_compress(const fmm_layout* layout, const void* farfield, int32_t first_group,
                                            int32_t count, double gamma, void* stream, fmm_tucker_t* inout) {
  clear_error();
  if (!inout) return fail(FMM_ERR_ARG, "inout is NULL");
  if (!(gamma >= 0.0 && gamma < 1.0)) return fail(FMM_ERR_ARG, "gamma must be in [0, 1)");
  Layout L;
  fmm_status st = copy_layout(layout, &L);
  if (st != FMM_OK) return st;
  if (first_group < 0 || count < 0 || (int64_t)first_group + count > L.n_groups)
    return fail(FMM_ERR_ARG, "group range outside the layout");
  if (*inout) {
    const Layout& H = (*inout)->layout;
    if (H.n_theta != L.n_theta || H.n_phi != L.n_phi || H.offsets != L.offsets)
      return fail(FMM_ERR_SHAPE, "layout differs from the handle's layout");
  }
  if (count == 0) {
    if (!*inout) return fmm_tucker_create(layout, inout);
    return FMM_OK;
  }
  if (!farfield) return fail(FMM_ERR_ARG, "farfield is NULL");
  if (reinterpret_cast<uintptr_t>(farfield) % 16) return fail(FMM_ERR_ARG, "farfield must be 16-byte aligned");
  if (!have_device()) return FMM_ERR_DEVICE;

  const int nt = L.n_theta, np = L.n_phi, nd = L.ndir();
  int nb_max = 0;
  for (int g = first_group; g < first_group + count; ++g) nb_max = std::max(nb_max, L.nb(g));
  const int64_t base_row = L.offsets[first_group];
  hipStream_t hs = static_cast<hipStream_t>(stream);

  BlasHandle bh;
  TFMM_BLAS(rocblas_create_handle(&bh.h));
  TFMM_BLAS(rocblas_set_stream(bh.h, hs));

  const size_t cz = sizeof(rocblas_double_complex);
  DevBuf s_tp, s_pt, gb, gt, gp, lam, work_e, info, vb, ut, up, y, z, cb;
  TFMM_HIP(s_tp.alloc(cz * (size_t)nb_max * nd));
  TFMM_HIP(s_pt.alloc(cz * (size_t)nb_max * nd));
  TFMM_HIP(gb.alloc(cz * (size_t)nb_max * nb_max));
  TFMM_HIP(gt.alloc(cz * (size_t)nt * nt));
  TFMM_HIP(gp.alloc(cz * (size_t)np * np));
  TFMM_HIP(lam.alloc(sizeof(double) * ((size_t)nb_max + nt + np)));
  TFMM_HIP(work_e.alloc(sizeof(double) * ((size_t)nb_max + nt + np)));
  TFMM_HIP(info.alloc(sizeof(rocblas_int) * 4));
  TFMM_HIP(vb.alloc(cz * (size_t)nb_max * nb_max));
  TFMM_HIP(ut.alloc(cz * (size_t)nt * nt));
  TFMM_HIP(up.alloc(cz * (size_t)np * np));
  TFMM_HIP(y.alloc(cz * (size_t)nd * nb_max));
  TFMM_HIP(z.alloc(cz * (size_t)nb_max * nt * np));
  TFMM_HIP(cb.alloc(cz * (size_t)nb_max * nt * np));

  bool created = false;
  if (!*inout) {
    st = fmm_tucker_create(layout, inout);
    if (st != FMM_OK) return st;
    created = true;
  }
  fmm_tucker_t h = *inout;
  auto bail = [&](fmm_status s) {
    if (created) {
      fmm_tucker_destroy(h);
      *inout = nullptr;
    }
    return s;
  };

  const double one = 1.0, zero = 0.0;
  const rocblas_double_complex cone = {1.0, 0.0}, czero = {0.0, 0.0};
  std::vector<double> lam_h((size_t)nb_max + nt + np);
  rocblas_int info_h[3];

  for (int g = first_group; g < first_group + count; ++g) {
    const int nb = L.nb(g);
    const int64_t row0 = L.offsets[g] - base_row;
    for (int alpha = 0; alpha < 2; ++alpha) {
      if (launch_gather_slab(farfield, row0, nb, alpha, nt, np, s_tp.p, s_pt.p, hs) != hipSuccess)
        return bail(fail(FMM_ERR_DEVICE, "gather kernel launch failed"));
      auto* A_tp = s_tp.as<rocblas_double_complex>();
      auto* A_pt = s_pt.as<rocblas_double_complex>();
      // Gram matrices (upper triangles)
      rocblas_status bs;
      bs = rocblas_zherk(bh.h, rocblas_fill_upper, rocblas_operation_conjugate_transpose, nb, nd, &one, A_tp, nd,
                         &zero, gb.as<rocblas_double_complex>(), nb);
      if (bs == rocblas_status_success)
        bs = rocblas_zherk(bh.h, rocblas_fill_upper, rocblas_operation_none, nt, nb * np, &one, A_pt, nt, &zero,
                           gt.as<rocblas_double_complex>(), nt);
      if (bs == rocblas_status_success)
        bs = rocblas_zherk(bh.h, rocblas_fill_upper, rocblas_operation_none, np, nb * nt, &one, A_tp, np, &zero,
                           gp.as<rocblas_double_complex>(), np);
      // eigendecompositions (ascending eigenvalues, eigenvectors in place)
      double* lb = lam.as<double>();
      double* lt = lb + nb_max;
      double* lp = lt + nt;
      double* ew = work_e.as<double>();
      rocblas_int* inf = info.as<rocblas_int>();
      if (bs == rocblas_status_success)
        bs = rocsolver_zheevd(bh.h, rocblas_evect_original, rocblas_fill_upper, nb, gb.as<rocblas_double_complex>(),
                              nb, lb, ew, inf);
      if (bs == rocblas_status_success)
        bs = rocsolver_zheevd(bh.h, rocblas_evect_original, rocblas_fill_upper, nt, gt.as<rocblas_double_complex>(),
                              nt, lt, ew, inf + 1);
      if (bs == rocblas_status_success)
        bs = rocsolver_zheevd(bh.h, rocblas_evect_original, rocblas_fill_upper, np, gp.as<rocblas_double_complex>(),
                              np, lp, ew, inf + 2);
      if (bs != rocblas_status_success)
        return bail(fail(FMM_ERR_DEVICE, "rocBLAS/rocSOLVER call failed for group %d: %s", g,
                         rocblas_status_to_string(bs)));
      if (hipMemcpyAsync(lam_h.data(), lb, sizeof(double) * ((size_t)nb_max + nt + np), hipMemcpyDeviceToHost, hs) !=
              hipSuccess ||
          hipMemcpyAsync(info_h, inf, sizeof(info_h), hipMemcpyDeviceToHost, hs) != hipSuccess ||
          hipStreamSynchronize(hs) != hipSuccess)
        return bail(fail(FMM_ERR_DEVICE, "eigenvalue copy failed"));
      if (info_h[0] != 0 || info_h[1] != 0 || info_h[2] != 0)
        return bail(fail(FMM_ERR_NUMERIC, "eigensolver did not converge for group %d polarisation %d", g, alpha));
      auto desc = [](const double* a, int n) {
        std::vector<double> v(n);
        for (int i = 0; i < n; ++i) v[i] = a[n - 1 - i];
        return v;
      };
      const std::vector<double> eb = desc(lam_h.data(), nb);
      const std::vector<double> et = desc(lam_h.data() + nb_max, nt);
      const std::vector<double> ep = desc(lam_h.data() + nb_max + nt, np);
      double norm2 = 0.0;
      for (double v : eb) norm2 += std::max(v, 0.0);
      for (double v : eb)
        if (!std::isfinite(v)) return bail(fail(FMM_ERR_NUMERIC, "non-finite far-field in group %d", g));
      const double thr2 = gamma * gamma / 3.0 * norm2;
      const int rb = truncation_rank(eb, thr2);
      const int rt = truncation_rank(et, thr2);
      const int rp = truncation_rank(ep, thr2);

      // leading eigenvectors, largest first
      if (launch_select_cols_rev(gb.p, nb, rb, vb.p, hs) != hipSuccess ||
          launch_select_cols_rev(gt.p, nt, rt, ut.p, hs) != hipSuccess ||
          launch_select_cols_rev(gp.p, np, rp, up.p, hs) != hipSuccess)
        return bail(fail(FMM_ERR_DEVICE, "column select launch failed"));
      // Y (nd x rb) = A^T conj(U^beta): the eigenvectors of conj(A A^H) are conj(U^beta)
      bs = rocblas_zgemm(bh.h, rocblas_operation_none, rocblas_operation_none, nd, rb, nb, &cone, A_tp, nd,
                         vb.as<rocblas_double_complex>(), nb, &czero, y.as<rocblas_double_complex>(), nd);
      // Z_b (r_theta x n_phi) = U^theta^H Y_b^T for every b
      if (bs == rocblas_status_success)
        bs = rocblas_zgemm_strided_batched(bh.h, rocblas_operation_conjugate_transpose, rocblas_operation_transpose,
                                           rt, np, nt, &cone, ut.as<rocblas_double_complex>(), nt, 0,
                                           y.as<rocblas_double_complex>(), np, nd, &czero,
                                           z.as<rocblas_double_complex>(), rt, (rocblas_stride)rt * np, rb);
      // C_b^T (r_phi x r_theta) = U^phi^H Z_b^T: row-major [theta'][phi'] per b
      if (bs == rocblas_status_success)
        bs = rocblas_zgemm_strided_batched(bh.h, rocblas_operation_conjugate_transpose, rocblas_operation_transpose,
                                           rp, rt, np, &cone, up.as<rocblas_double_complex>(), np, 0,
                                           z.as<rocblas_double_complex>(), rt, (rocblas_stride)rt * np, &czero,
                                           cb.as<rocblas_double_complex>(), rp, (rocblas_stride)rt * rp, rb);
      if (bs != rocblas_status_success)
        return bail(fail(FMM_ERR_DEVICE, "core projection failed for group %d: %s", g, rocblas_status_to_string(bs)));

      TensorFactors tf;
      tf.rt = rt;
      tf.rp = rp;
      tf.rb = rb;
      std::vector<cd> vb_h((size_t)nb * rb), ut_h((size_t)nt * rt), up_h((size_t)np * rp), cb_h((size_t)rb * rt * rp);
      if (hipMemcpyAsync(vb_h.data(), vb.p, cz * vb_h.size(), hipMemcpyDeviceToHost, hs) != hipSuccess ||
          hipMemcpyAsync(ut_h.data(), ut.p, cz * ut_h.size(), hipMemcpyDeviceToHost, hs) != hipSuccess ||
          hipMemcpyAsync(up_h.data(), up.p, cz * up_h.size(), hipMemcpyDeviceToHost, hs) != hipSuccess ||
          hipMemcpyAsync(cb_h.data(), cb.p, cz * cb_h.size(), hipMemcpyDeviceToHost, hs) != hipSuccess ||
          hipStreamSynchronize(hs) != hipSuccess)
        return bail(fail(FMM_ERR_DEVICE, "factor copy failed"));
      tf.ub.resize((size_t)nb * rb);
      for (int n = 0; n < nb; ++n)
        for (int b = 0; b < rb; ++b) tf.ub[(size_t)n * rb + b] = std::conj(vb_h[(size_t)b * nb + n]);
      tf.ut.resize((size_t)nt * rt);
      for (int i = 0; i < nt; ++i)
        for (int a = 0; a < rt; ++a) tf.ut[(size_t)i * rt + a] = ut_h[(size_t)a * nt + i];
      tf.up.resize((size_t)np * rp);
      for (int j = 0; j < np; ++j)
        for (int c = 0; c < rp; ++c) tf.up[(size_t)j * rp + c] = up_h[(size_t)c * np + j];
      tf.core.resize((size_t)rt * rp * rb);
      for (int b = 0; b < rb; ++b)
        for (int a = 0; a < rt; ++a)
          for (int c = 0; c < rp; ++c)
            tf.core[((size_t)a * rp + c) * rb + b] = cb_h[(size_t)b * rt * rp + (size_t)a * rp + c];
      h->t[2 * (size_t)g + alpha] = std::move(tf);
    }
  }
  for (auto& s : h->slot) s.ready = false;
  return FMM_OK;
}
