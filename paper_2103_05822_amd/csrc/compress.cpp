// Setup: truncated HOSVD of the dense far-field tensors (Section II.B, eq. (6)),
// FP64 on the device; and the truncated SVD of the basis mode alone, the paper's
// comparison method.
//
// For each (group, polarisation) tensor A (n_theta x n_phi x n_beta):
//   1. the Gram matrices of the three mode unfoldings: the basis mode with rocBLAS
//      ZHERK, the two angular modes with mode_gram (a tall-skinny reduction that
//      ZHERK handles poorly);
//   2. their Hermitian eigendecompositions with rocSOLVER ZHEEVD: eigenvectors are
//      the left singular vectors of the unfoldings, eigenvalues the squared
//      singular values;
//   3. per mode, the energy the tensor keeps along every eigenvector, ||u_i^H A_(p)||^2,
//      from the projections themselves (a ZGEMM and a reduction): the Gram
//      eigenvalues carry absolute errors near eps s_max^2 each, which summed over a
//      long tail would swamp the threshold at small gamma, while the projected
//      energies are sums of squares of accurately computed entries;
//   4. per mode, the smallest rank whose discarded tail satisfies
//      sum_{i>=r} e_i <= gamma^2/3 ||A||_F^2 (host, FP64), which bounds the mode's
//      projection error exactly;
//   5. the core C = A x_3 U^beta* x_1 U^theta* x_2 U^phi* with three ZGEMMs.
// The eigensolver is latency-bound for these sizes, so tensors are spread over
// several worker threads, each with its own stream, rocBLAS handle and workspace.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <thread>

#include "internal.hpp"
#include "kernels.hpp"

using namespace tuckfmm;

namespace {

// Worker threads of the HOSVD driver (TUCKFMM_COMPRESS_WORKERS overrides; 1 runs the
// tensors one after another on one stream).
int worker_count() {
  const char* e = std::getenv("TUCKFMM_COMPRESS_WORKERS");
  const int n = e ? std::atoi(e) : 8;
  return std::min(std::max(n, 1), 32);
}

// Smallest r >= 1 with sum_{i >= r} lam_desc[i] <= thr2 (lam sorted descending);
// thr2 <= 0 keeps everything.
int truncation_rank(const std::vector<double>& lam_desc, double thr2) {
  const int n = (int)lam_desc.size();
  if (thr2 <= 0.0) return n;
  double tail = 0.0;
  int r = n;
  for (int i = n - 1; i >= 1; --i) {
    tail += std::max(lam_desc[i], 0.0);
    if (tail <= thr2)
      r = i;
    else
      break;
  }
  return std::max(r, 1);
}

struct Shared {
  std::mutex mu;
  fmm_status status = FMM_OK;
  std::string message;
  std::atomic<int> next{0};
  void error(fmm_status st, const std::string& msg) {
    std::lock_guard<std::mutex> lk(mu);
    if (status == FMM_OK) {
      status = st;
      message = msg;
    }
  }
  bool failed() {
    std::lock_guard<std::mutex> lk(mu);
    return status != FMM_OK;
  }
};

struct Worker {
  hipStream_t s = nullptr;
  rocblas_handle h = nullptr;
  void* buf[9] = {};
  ~Worker() {
    for (void* p : buf)
      if (p) (void)hipFree(p);
    if (h) rocblas_destroy_handle(h);
    if (s) (void)hipStreamDestroy(s);
  }
};

struct Job {
  const Layout* L;
  const void* farfield;
  int64_t base_row;
  int first_group;
  int n_tensors;
  int nb_max;
  double gamma;
  bool svd;  // truncated SVD of the basis mode only (the paper's comparison method)
  fmm_tucker_s* handle;
};

std::string hip_msg(const char* what, hipError_t e) { return std::string(what) + ": " + hipGetErrorString(e); }

// The FP64 scratch of one worker (buf[4]): eigenvalues, eigensolver work, the
// projected energies (each nbm + nt + np doubles: basis, theta, phi modes) and the
// eigensolver's three info words.
struct Scalars {
  double *lb, *lt, *lp, *ework, *eb, *et, *ep;
  rocblas_int* info;
  Scalars(void* buf, int nbm, int nt, int np) {
    lb = static_cast<double*>(buf);
    lt = lb + nbm;
    lp = lt + nt;
    ework = lp + np;
    eb = ework + nbm + nt + np;
    et = eb + nbm;
    ep = et + nt;
    info = reinterpret_cast<rocblas_int*>(ep + np);
  }
  static size_t bytes(int nbm, int nt, int np) { return sizeof(double) * 3 * ((size_t)nbm + nt + np) + 64; }
};

// The tensor's per-basis-function energies (row sums of |A|^2, into `tmp`, nb doubles),
// checked on the host before any eigensolver sees the data: a NaN or Inf far-field
// is reported, not decomposed.
std::string check_finite(Worker& w, const void* slab, int nb, int nd, double* tmp) {
  hipError_t he = launch_strided_energy(slab, nb, nd, nd, 1, tmp, w.s);
  if (he != hipSuccess) return hip_msg("energy kernel", he);
  std::vector<double> e(nb);
  if ((he = hipMemcpyAsync(e.data(), tmp, sizeof(double) * nb, hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipStreamSynchronize(w.s)) != hipSuccess)
    return hip_msg("energy copy", he);
  for (double v : e)
    if (!std::isfinite(v)) return "NUMERIC:non-finite far-field values";
  return std::string();
}

// Reversed copy: ascending eigenvalue order -> descending.
std::vector<double> reversed(const double* a, int n) {
  std::vector<double> v(n);
  for (int i = 0; i < n; ++i) v[i] = a[n - 1 - i];
  return v;
}

// Truncated SVD of tensor t (basis mode only): U^beta from the basis-mode Gram matrix,
// rank rule sqrt(sum_{i>=r} s_i^2) <= gamma ||A||_F, W = A conj(U^beta) (N_dir x r_beta).
// Stored as a Tucker item with identity angular factors and core W.
std::string decompose_svd(const Job& J, Worker& w, int t) {
  const Layout& L = *J.L;
  const int g = J.first_group + t / 2, alpha = t % 2;
  const int nt = L.n_theta, np = L.n_phi, nd = L.ndir();
  const int nb = L.nb(g);
  const int64_t row0 = L.offsets[g] - J.base_row;
  using Z = rocblas_double_complex;
  Z* slab = static_cast<Z*>(w.buf[0]);
  Z* gb = static_cast<Z*>(w.buf[1]);
  const Scalars sc(w.buf[4], J.nb_max, nt, np);
  double* lb = sc.lb;
  Z* vb = static_cast<Z*>(w.buf[6]);
  Z* y = static_cast<Z*>(w.buf[7]);
  double* ework = sc.ework;
  rocblas_int* info = sc.info;

  hipError_t he = launch_gather_slab(J.farfield, row0, nb, alpha, nt, np, slab, nullptr, w.s);
  if (he != hipSuccess) return hip_msg("gather kernel", he);
  {
    const std::string bad = check_finite(w, slab, nb, nd, sc.eb);
    if (!bad.empty()) return bad;
  }
  const double one = 1.0, zero = 0.0;
  const Z cone = {1.0, 0.0}, czero = {0.0, 0.0};
  rocblas_status bs = rocblas_status_success;
  std::vector<double> en_h(nb);
  // divide and conquer first, QR iteration if the eigenvectors come back non-finite
  for (int attempt = 0;; ++attempt) {
    bs = rocblas_zherk(w.h, rocblas_fill_upper, rocblas_operation_conjugate_transpose, nb, nd, &one, slab, nd, &zero,
                       gb, nb);
    if (bs != rocblas_status_success) return std::string("zherk: ") + rocblas_status_to_string(bs);
    bs = attempt ? rocsolver_zheev(w.h, rocblas_evect_original, rocblas_fill_upper, nb, gb, nb, lb, ework, info)
                 : rocsolver_zheevd(w.h, rocblas_evect_original, rocblas_fill_upper, nb, gb, nb, lb, ework, info);
    if (bs != rocblas_status_success) return std::string("eigensolver: ") + rocblas_status_to_string(bs);
    // energy along every eigenvector: column norms of A^T conj(U^beta) over all columns
    bs = rocblas_zgemm(w.h, rocblas_operation_none, rocblas_operation_none, nd, nb, nb, &cone, slab, nd, gb, nb,
                       &czero, y, nd);
    if (bs != rocblas_status_success) return std::string("energy projection: ") + rocblas_status_to_string(bs);
    if ((he = launch_strided_energy(y, nb, nd, nd, 1, sc.eb, w.s)) != hipSuccess) return hip_msg("energy kernel", he);
    rocblas_int info_h = 0;
    if ((he = hipMemcpyAsync(en_h.data(), sc.eb, sizeof(double) * nb, hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
        (he = hipMemcpyAsync(&info_h, info, sizeof(info_h), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
        (he = hipStreamSynchronize(w.s)) != hipSuccess)
      return hip_msg("energy copy", he);
    if (info_h != 0) return "NUMERIC:eigensolver did not converge";
    bool ok = true;
    for (double v : en_h) ok = ok && std::isfinite(v);
    if (ok) break;
    if (attempt > 0) return "NUMERIC:non-finite far-field values or eigenvectors";
  }
  const std::vector<double> eb = reversed(en_h.data(), nb);
  double norm2 = 0.0;
  for (double v : eb) norm2 += v;
  if (!std::isfinite(norm2)) return "NUMERIC:non-finite far-field values";
  const int rb = truncation_rank(eb, J.gamma * J.gamma * norm2);
  if ((he = launch_select_cols_rev(gb, nb, rb, vb, w.s)) != hipSuccess) return hip_msg("column select kernel", he);
  // W (nd x rb) = A conj(U^beta): as in the HOSVD, the Gram eigenvectors are conj(U^beta)
  bs = rocblas_zgemm(w.h, rocblas_operation_none, rocblas_operation_none, nd, rb, nb, &cone, slab, nd, vb, nb,
                     &czero, y, nd);
  if (bs != rocblas_status_success) return std::string("W projection: ") + rocblas_status_to_string(bs);
  std::vector<cd> vb_h((size_t)nb * rb), w_h((size_t)nd * rb);
  const size_t cz = sizeof(Z);
  if ((he = hipMemcpyAsync(vb_h.data(), vb, cz * vb_h.size(), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipMemcpyAsync(w_h.data(), y, cz * w_h.size(), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipStreamSynchronize(w.s)) != hipSuccess)
    return hip_msg("factor copy", he);
  TensorFactors tf;
  tf.rt = nt;
  tf.rp = np;
  tf.rb = rb;
  tf.ident = true;
  tf.ub.resize((size_t)nb * rb);
  for (int n = 0; n < nb; ++n)
    for (int b = 0; b < rb; ++b) tf.ub[(size_t)n * rb + b] = std::conj(vb_h[(size_t)b * nb + n]);
  tf.ut.assign((size_t)nt * nt, cd(0.0, 0.0));
  for (int i = 0; i < nt; ++i) tf.ut[(size_t)i * nt + i] = cd(1.0, 0.0);
  tf.up.assign((size_t)np * np, cd(0.0, 0.0));
  for (int j = 0; j < np; ++j) tf.up[(size_t)j * np + j] = cd(1.0, 0.0);
  tf.core.resize((size_t)nd * rb);  // [theta][phi][rb]: direction i = theta * n_phi + phi
  for (int i = 0; i < nd; ++i)
    for (int b = 0; b < rb; ++b) tf.core[(size_t)i * rb + b] = w_h[(size_t)b * nd + i];
  J.handle->t[2 * (size_t)g + alpha] = std::move(tf);
  return std::string();
}

// Decompose tensor t of the job on worker w.  Returns an empty string on success.
std::string decompose(const Job& J, Worker& w, int t) {
  if (J.svd) return decompose_svd(J, w, t);
  const Layout& L = *J.L;
  const int g = J.first_group + t / 2, alpha = t % 2;
  const int nt = L.n_theta, np = L.n_phi, nd = L.ndir();
  const int nb = L.nb(g);
  const int64_t row0 = L.offsets[g] - J.base_row;
  using Z = rocblas_double_complex;
  Z* slab = static_cast<Z*>(w.buf[0]);
  Z* gb = static_cast<Z*>(w.buf[1]);
  Z* gt = static_cast<Z*>(w.buf[2]);
  Z* gp = static_cast<Z*>(w.buf[3]);
  const Scalars sc(w.buf[4], J.nb_max, nt, np);
  Z* part = static_cast<Z*>(w.buf[5]);
  Z* vb = static_cast<Z*>(w.buf[6]);
  Z* y = static_cast<Z*>(w.buf[7]);
  Z* z = static_cast<Z*>(w.buf[8]);
  Z* ut = gt + (size_t)nt * nt;  // selected columns live after each Gram matrix
  Z* up = gp + (size_t)np * np;
  double *lb = sc.lb, *lt = sc.lt, *lp = sc.lp, *ework = sc.ework;
  rocblas_int* info = sc.info;

  hipError_t he = launch_gather_slab(J.farfield, row0, nb, alpha, nt, np, slab, nullptr, w.s);
  if (he != hipSuccess) return hip_msg("gather kernel", he);
  {
    const std::string bad = check_finite(w, slab, nb, nd, sc.eb);
    if (!bad.empty()) return bad;
  }
  const double one = 1.0, zero = 0.0;
  const Z cone = {1.0, 0.0}, czero = {0.0, 0.0};
  rocblas_status bs = rocblas_status_success;
  std::vector<double> en_h((size_t)J.nb_max + nt + np);
  // Two attempts: the divide-and-conquer eigensolver, then, for a mode whose
  // eigenvectors came back non-finite (seen with an exactly zero row in the
  // unfolding, e.g. the phi pattern of a plate at phi = 0), QR iteration.
  bool qr_b = false, qr_ang = false;
  for (int attempt = 0;; ++attempt) {
    const bool do_b = attempt == 0 || qr_b, do_ang = attempt == 0 || qr_ang;
    if (do_b) {
      bs = rocblas_zherk(w.h, rocblas_fill_upper, rocblas_operation_conjugate_transpose, nb, nd, &one, slab, nd,
                         &zero, gb, nb);
      if (bs != rocblas_status_success) return std::string("zherk: ") + rocblas_status_to_string(bs);
      bs = qr_b ? rocsolver_zheev(w.h, rocblas_evect_original, rocblas_fill_upper, nb, gb, nb, lb, ework, info)
                : rocsolver_zheevd(w.h, rocblas_evect_original, rocblas_fill_upper, nb, gb, nb, lb, ework, info);
      if (bs != rocblas_status_success) return std::string("eigensolver: ") + rocblas_status_to_string(bs);
    }
    if (do_ang) {
      if ((he = launch_mode_gram(slab, nb, nt, np, part, gt, gp, w.s)) != hipSuccess)
        return hip_msg("mode_gram kernel", he);
      auto heev = qr_ang ? rocsolver_zheev : rocsolver_zheevd;
      bs = heev(w.h, rocblas_evect_original, rocblas_fill_upper, nt, gt, nt, lt, ework, info + 1);
      if (bs == rocblas_status_success)
        bs = heev(w.h, rocblas_evect_original, rocblas_fill_upper, np, gp, np, lp, ework, info + 2);
      if (bs != rocblas_status_success) return std::string("eigensolver: ") + rocblas_status_to_string(bs);
    }

    // energy along every eigenvector of each mode, from the projections:
    //   basis: column norms of Y = A^T conj(U^beta) (all columns);
    //   theta: row norms of U^theta^H S_b over all b;  phi: row norms of U^phi^H S_b^T
    bs = rocblas_zgemm(w.h, rocblas_operation_none, rocblas_operation_none, nd, nb, nb, &cone, slab, nd, gb, nb,
                       &czero, y, nd);
    if (bs != rocblas_status_success) return std::string("energy projection: ") + rocblas_status_to_string(bs);
    if ((he = launch_strided_energy(y, nb, nd, nd, 1, sc.eb, w.s)) != hipSuccess) return hip_msg("energy kernel", he);
    bs = rocblas_zgemm_strided_batched(w.h, rocblas_operation_conjugate_transpose, rocblas_operation_transpose, nt,
                                       np, nt, &cone, gt, nt, 0, slab, np, nd, &czero, z, nt, (rocblas_stride)nt * np,
                                       nb);
    if (bs != rocblas_status_success) return std::string("energy projection: ") + rocblas_status_to_string(bs);
    if ((he = launch_strided_energy(z, nt, 1, (int64_t)np * nb, nt, sc.et, w.s)) != hipSuccess)
      return hip_msg("energy kernel", he);
    bs = rocblas_zgemm_strided_batched(w.h, rocblas_operation_conjugate_transpose, rocblas_operation_none, np, nt, np,
                                       &cone, gp, np, 0, slab, np, nd, &czero, z, np, (rocblas_stride)np * nt, nb);
    if (bs != rocblas_status_success) return std::string("energy projection: ") + rocblas_status_to_string(bs);
    if ((he = launch_strided_energy(z, np, 1, (int64_t)nt * nb, np, sc.ep, w.s)) != hipSuccess)
      return hip_msg("energy kernel", he);

    rocblas_int info_h[3];
    if ((he = hipMemcpyAsync(en_h.data(), sc.eb, sizeof(double) * en_h.size(), hipMemcpyDeviceToHost, w.s)) !=
            hipSuccess ||
        (he = hipMemcpyAsync(info_h, info, sizeof(info_h), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
        (he = hipStreamSynchronize(w.s)) != hipSuccess)
      return hip_msg("energy copy", he);
    if (info_h[0] != 0 || info_h[1] != 0 || info_h[2] != 0) return "NUMERIC:eigensolver did not converge";
    auto finite = [&](size_t off, int n) {
      for (int i = 0; i < n; ++i)
        if (!std::isfinite(en_h[off + i])) return false;
      return true;
    };
    const bool ok_b = finite(0, nb);
    const bool ok_ang = finite(J.nb_max, nt) && finite((size_t)J.nb_max + nt, np);
    if (ok_b && ok_ang) break;
    if (attempt > 0) return "NUMERIC:non-finite far-field values or eigenvectors";
    qr_b = !ok_b;
    qr_ang = !ok_ang;
  }
  const std::vector<double> eb = reversed(en_h.data(), nb);
  const std::vector<double> et = reversed(en_h.data() + J.nb_max, nt);
  const std::vector<double> ep = reversed(en_h.data() + J.nb_max + nt, np);
  double norm2 = 0.0;
  for (double v : eb) norm2 += v;
  if (!std::isfinite(norm2)) return "NUMERIC:non-finite far-field values";
  const double thr2 = J.gamma * J.gamma / 3.0 * norm2;
  const int rb = truncation_rank(eb, thr2);
  const int rt = truncation_rank(et, thr2);
  const int rp = truncation_rank(ep, thr2);

  if ((he = launch_select_cols_rev(gb, nb, rb, vb, w.s)) != hipSuccess ||
      (he = launch_select_cols_rev(gt, nt, rt, ut, w.s)) != hipSuccess ||
      (he = launch_select_cols_rev(gp, np, rp, up, w.s)) != hipSuccess)
    return hip_msg("column select kernel", he);
  // Y (nd x rb) = A^T conj(U^beta); the eigenvectors of conj(A A^H) are conj(U^beta)
  bs = rocblas_zgemm(w.h, rocblas_operation_none, rocblas_operation_none, nd, rb, nb, &cone, slab, nd, vb, nb,
                     &czero, y, nd);
  // Z_b (r_theta x n_phi) = U^theta^H Y_b^T for every b
  if (bs == rocblas_status_success)
    bs = rocblas_zgemm_strided_batched(w.h, rocblas_operation_conjugate_transpose, rocblas_operation_transpose, rt,
                                       np, nt, &cone, ut, nt, 0, y, np, nd, &czero, z, rt, (rocblas_stride)rt * np, rb);
  // C_b^T (r_phi x r_theta) = U^phi^H Z_b^T, i.e. row-major [theta'][phi'] per b; reuse slab
  Z* cb = slab;
  if (bs == rocblas_status_success)
    bs = rocblas_zgemm_strided_batched(w.h, rocblas_operation_conjugate_transpose, rocblas_operation_transpose, rp,
                                       rt, np, &cone, up, np, 0, z, rt, (rocblas_stride)rt * np, &czero, cb, rp,
                                       (rocblas_stride)rt * rp, rb);
  if (bs != rocblas_status_success) return std::string("core projection: ") + rocblas_status_to_string(bs);

  std::vector<cd> vb_h((size_t)nb * rb), ut_h((size_t)nt * rt), up_h((size_t)np * rp), cb_h((size_t)rb * rt * rp);
  const size_t cz = sizeof(Z);
  if ((he = hipMemcpyAsync(vb_h.data(), vb, cz * vb_h.size(), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipMemcpyAsync(ut_h.data(), ut, cz * ut_h.size(), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipMemcpyAsync(up_h.data(), up, cz * up_h.size(), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipMemcpyAsync(cb_h.data(), cb, cz * cb_h.size(), hipMemcpyDeviceToHost, w.s)) != hipSuccess ||
      (he = hipStreamSynchronize(w.s)) != hipSuccess)
    return hip_msg("factor copy", he);
  TensorFactors tf;
  tf.rt = rt;
  tf.rp = rp;
  tf.rb = rb;
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
  J.handle->t[2 * (size_t)g + alpha] = std::move(tf);
  return std::string();
}

std::string setup_worker(Worker& w, const Job& J, int device) {
  hipError_t he = hipSetDevice(device);
  if (he != hipSuccess) return hip_msg("hipSetDevice", he);
  if ((he = hipStreamCreateWithFlags(&w.s, hipStreamNonBlocking)) != hipSuccess) return hip_msg("stream", he);
  rocblas_status bs = rocblas_create_handle(&w.h);
  if (bs == rocblas_status_success) bs = rocblas_set_stream(w.h, w.s);
  if (bs != rocblas_status_success) return std::string("rocblas handle: ") + rocblas_status_to_string(bs);
  const int nt = J.L->n_theta, np = J.L->n_phi, nd = J.L->ndir();
  const size_t nbm = (size_t)J.nb_max;
  const size_t cz = 16;
  const size_t sizes[9] = {
      cz * nbm * nd,                                               // slab (also the core output)
      cz * nbm * nbm,                                              // basis-mode Gram / eigenvectors
      cz * (size_t)nt * nt * 2,                                    // theta Gram + selected columns
      cz * (size_t)np * np * 2,                                    // phi Gram + selected columns
      Scalars::bytes((int)nbm, nt, np),                            // eigenvalues, work, energies, info
      cz * (size_t)mode_gram_chunks(J.nb_max) * (nt * nt + np * np),  // Gram partials
      cz * nbm * nbm,                                              // selected basis-mode columns
      cz * (size_t)nd * nbm,                                       // Y
      cz * nbm * nd,                                               // Z
  };
  for (int i = 0; i < 9; ++i)
    if ((he = hipMalloc(&w.buf[i], sizes[i])) != hipSuccess) return hip_msg("workspace hipMalloc", he);
  return std::string();
}

}  // namespace

namespace {
fmm_status compress_impl(const fmm_layout* layout, const void* farfield, int32_t first_group, int32_t count,
                         double gamma, void* stream, fmm_tucker_t* inout, bool svd) {
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
  if (count == 0) return *inout ? FMM_OK : fmm_tucker_create(layout, inout);
  if (!farfield) return fail(FMM_ERR_ARG, "farfield is NULL");
  if (reinterpret_cast<uintptr_t>(farfield) % 16) return fail(FMM_ERR_ARG, "farfield must be 16-byte aligned");
  if (!have_device()) return FMM_ERR_DEVICE;
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));
  {
    int lim = 0;
    TFMM_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if ((size_t)16 * L.n_theta * L.n_phi > (size_t)lim)
      return fail(FMM_ERR_UNSUPPORTED, "angular grid %dx%d too large for the Gram kernel's LDS", L.n_theta, L.n_phi);
  }
  // the far-field may still be in flight on the caller's stream
  TFMM_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));

  bool created = false;
  if (!*inout) {
    st = fmm_tucker_create(layout, inout);
    if (st != FMM_OK) return st;
    created = true;
  }
  Job J;
  J.L = &L;
  J.farfield = farfield;
  J.base_row = L.offsets[first_group];
  J.first_group = first_group;
  J.n_tensors = 2 * count;
  J.nb_max = 0;
  for (int g = first_group; g < first_group + count; ++g) J.nb_max = std::max(J.nb_max, L.nb(g));
  J.gamma = gamma;
  J.svd = svd;
  J.handle = *inout;

  Shared sh;
  const int nw = std::min(worker_count(), J.n_tensors);
  std::vector<std::thread> pool;
  for (int i = 0; i < nw; ++i)
    pool.emplace_back([&]() {
      Worker w;
      std::string msg = setup_worker(w, J, dev);
      if (!msg.empty()) {
        sh.error(FMM_ERR_DEVICE, msg);
        return;
      }
      for (;;) {
        const int t = sh.next.fetch_add(1);
        if (t >= J.n_tensors || sh.failed()) break;
        msg = decompose(J, w, t);
        if (!msg.empty()) {
          const bool numeric = msg.rfind("NUMERIC:", 0) == 0;
          sh.error(numeric ? FMM_ERR_NUMERIC : FMM_ERR_DEVICE,
                   "group " + std::to_string(J.first_group + t / 2) + " polarisation " + std::to_string(t % 2) +
                       ": " + (numeric ? msg.substr(8) : msg));
          break;
        }
      }
      (void)hipStreamSynchronize(w.s);
    });
  for (auto& th : pool) th.join();
  if (sh.status != FMM_OK) {
    if (created) {
      fmm_tucker_destroy(*inout);
      *inout = nullptr;
    }
    return fail(sh.status, "%s", sh.message.c_str());
  }
  for (auto& s : (*inout)->slot) s.ready = false;
  return FMM_OK;
}
}  // namespace

extern "C" fmm_status fmm_farfield_compress(const fmm_layout* layout, const void* farfield, int32_t first_group,
                                            int32_t count, double gamma, void* stream, fmm_tucker_t* inout) {
  clear_error();
  return compress_impl(layout, farfield, first_group, count, gamma, stream, inout, false);
}

extern "C" fmm_status fmm_farfield_compress_svd(const fmm_layout* layout, const void* farfield, int32_t first_group,
                                                int32_t count, double gamma, void* stream, fmm_tucker_t* inout) {
  clear_error();
  return compress_impl(layout, farfield, first_group, count, gamma, stream, inout, true);
}
