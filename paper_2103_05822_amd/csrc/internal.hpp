// Host-side runtime of the library: handle types, error reporting, validation.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "tuckfmm.h"
#include "desc.hpp"

namespace tuckfmm {

using cd = std::complex<double>;

// Records the message for fmm_last_error() and returns `st`.
fmm_status fail(fmm_status st, const char* fmt, ...);
void clear_error();
const char* last_error_cstr();

// True if at least one HIP device is present (records FMM_ERR_DEVICE otherwise).
bool have_device();

#define TFMM_HIP(expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::tuckfmm::fail(FMM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Validated copy of a layout.
struct Layout {
  int32_t n_theta = 0, n_phi = 0, n_groups = 0;
  std::vector<int64_t> offsets;
  int64_t n_basis() const { return offsets.empty() ? 0 : offsets.back(); }
  int32_t nb(int g) const { return (int32_t)(offsets[g + 1] - offsets[g]); }
  int32_t ndir() const { return n_theta * n_phi; }
};
fmm_status copy_layout(const fmm_layout* in, Layout* out);

struct TensorFactors {
  int32_t rt = 0, rp = 0, rb = 0;
  std::vector<cd> core;  // paper shape [rt][rp][rb]
  std::vector<cd> ut;    // [n_theta][rt]
  std::vector<cd> up;    // [n_phi][rp]
  std::vector<cd> ub;    // [nb][rb]
  bool set() const { return rt > 0; }
};

struct PrecSlot {
  bool ready = false;
  char* arena = nullptr;   // caller-owned device memory
  size_t bytes = 0;
  int device = -1;
  TuckPlan plan;          // device pointers into the arena
};

}  // namespace tuckfmm

struct fmm_tucker_s {
  tuckfmm::Layout layout;
  std::vector<tuckfmm::TensorFactors> t;  // [n_groups * 2], index 2g + alpha
  tuckfmm::PrecSlot slot[4];
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

struct fmm_dense_s {
  tuckfmm::Layout layout;
  int device = -1;
  tuckfmm::DenseGroup* d_groups = nullptr;  // library-owned device table
  int64_t* d_offsets = nullptr;
};

struct fmm_geometry_s {
  int64_t n_verts = 0, n_tris = 0;
  std::vector<double> verts;  // [n_verts][3]
  std::vector<int32_t> tris;  // [n_tris][3]
  double origin[3] = {0, 0, 0};
  double box = 0.0;
  int32_t K = 0;
  double k = 0.0;
  int32_t n_theta = 0, n_phi = 0;
  // group-ordered basis functions
  std::vector<int64_t> perm;      // edge number of each basis function
  std::vector<int32_t> tri_p, tri_m, free_p, free_m;
  std::vector<double> length;
  std::vector<int64_t> offsets;   // [G+1]
  std::vector<double> centers;    // [G][3]
  std::vector<double> theta, phi; // grid
  std::vector<double> dirs;       // [ndir][9]: k_hat, theta_hat, phi_hat
  // device copies for fmm_farfield_fill
  int device = -1;
  double* d_rowdata = nullptr;
  double* d_dirs = nullptr;
};
