// Host-side runtime of the library: handle types, error reporting, validation.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdarg>
#include <cstdint>
#include <list>
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
  bool ident = false;    // U^theta and U^phi are identities (truncated-SVD method)
  std::vector<cd> core;  // paper shape [rt][rp][rb]
  std::vector<cd> ut;    // [n_theta][rt]
  std::vector<cd> up;    // [n_phi][rp]
  std::vector<cd> ub;    // [nb][rb]
  bool set() const { return rt > 0; }
};

// One chunk of right-hand sides of the multi-RHS path (columns r0 .. r0 + rc - 1).
// Launch j (0..3) of a stage computes contraction j of every item; the aggregation,
// disaggregation and merged pass tile lists index the chunk's problem table.
struct MrhsChunk {
  int r0 = 0, rc = 0;
  const CGemm* probs = nullptr;         // device
  const CTile* tiles[3][4] = {};        // [agg, dis, pass][launch], device
  int n_tiles[3][4] = {};
};

// Library-owned device tables and scratch of the multi-RHS path for one nrhs.
struct MrhsPlan {
  int nrhs = 0;
  int rhs_chunk = 0;   // columns per chunk
  int tile_steps = 0;  // K steps a workgroup aims to run (column blocks per tile)
  int order = 0;       // angular contraction order: 0 each item's cheaper, 1 theta first, 2 phi first
  char* dev = nullptr;  // one allocation: problem tables, tile lists, scratch
  size_t dev_bytes = 0;
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  std::vector<MrhsChunk> chunks;
};

// Tuned choice for one nrhs: path 0 = streaming kernels (workgroup size `threads`),
// 1 = matrix-core products (K steps per tile, right-hand sides per chunk, angular
// contraction order).
struct TuneChoice {
  int nrhs = 0, path = 0, tile_steps = 0, rhs_chunk = 0, threads = 0, order = 0;
};

struct PrecSlot {
  bool ready = false;
  char* arena = nullptr;   // caller-owned device memory
  size_t bytes = 0;
  int device = -1;
  TuckPlan plan;          // device pointers into the arena
  std::vector<TuckItem> items;      // host copy of the item table
  int threads = 512;                // default workgroup size of the streaming kernels
  bool streams = true;              // the streaming kernels' LDS fits the largest item
  std::list<MrhsPlan> mrhs;         // built on first use per (nrhs, knobs); stable addresses
  std::vector<TuneChoice> tuned;
  void* part = nullptr;             // library-owned partial sums of split items (device)
  size_t part_bytes = 0;
  int32_t* next = nullptr;          // library-owned work counter of the pass kernel (device)
};

// Multi-RHS path (mrhs_plan.cpp).
constexpr int kMrhsDefaultSteps = 16;
constexpr int kMrhsDefaultChunk = 64;
// Host image of the tables: problems [8][n_items] (product j of item i at j n_items + i)
// and tile lists [agg, dis, pass][launch] per chunk; scratch offsets in complex elements.
struct MrhsHostChunk {
  int r0 = 0, rc = 0;
  std::vector<CGemm> probs;
  std::vector<CTile> lists[3][4];
};
struct MrhsHost {
  int64_t scratch_elems = 0;
  std::vector<MrhsHostChunk> chunks;
};
void mrhs_build_host(const std::vector<TuckItem>& items, const Layout& L, int nrhs, int tile_steps, int rhs_chunk,
                     int order, MrhsHost* out);
// Plan for (slot, nrhs) with the given knobs (0 = defaults), built on first use.
// elem_bytes: 8 (complex64 slot) or 16 (complex128 slot), the size of a scratch value.
fmm_status mrhs_get(PrecSlot& s, size_t elem_bytes, const Layout& L, int nrhs, int tile_steps, int rhs_chunk,
                    int order, MrhsPlan** out);
// stage: 0 aggregation, 1 disaggregation, 2 both (merged launches).
fmm_status mrhs_run(const MrhsPlan& p, const PrecSlot& s, int variant, size_t elem_bytes, int stage, const void* x,
                    void* F, const void* G, void* V, hipStream_t st);
void mrhs_free(MrhsPlan& p);
void mrhs_release(PrecSlot& s);

}  // namespace tuckfmm

struct fmm_tucker_s;
namespace tuckfmm {
// The pass of fmm_tucker_pass on the streaming kernels with the split items' partial
// sums in `scratch` (device memory of scratch_bytes) instead of the handle's buffer:
// validates, checks the size, launches; allocates nothing.
fmm_status noalloc_pass(fmm_tucker_s* h, fmm_prec prec, int32_t nrhs, const void* x, void* F, const void* G,
                        void* V, hipStream_t hs, void* scratch, size_t scratch_bytes);
}  // namespace tuckfmm

struct fmm_tucker_s {
  tuckfmm::Layout layout;
  std::vector<tuckfmm::TensorFactors> t;  // [n_groups * 2], index 2g + alpha
  // box grid of F and G (eq. (3)): K boxes, box[g] the box of group g; empty: the
  // group-compact layout [n_groups][2]
  int64_t n_boxes = 0;
  int32_t box_dims[3] = {0, 0, 0};
  std::vector<int64_t> box;
  tuckfmm::PrecSlot slot[4];
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

struct fmm_dense_s {
  tuckfmm::Layout layout;
  int device = -1;
  tuckfmm::DenseGroup* d_groups = nullptr;  // library-owned device table
  int64_t* d_offsets = nullptr;
  tuckfmm::DenseBlock* d_blocks = nullptr;  // row blocks, in XCD order (see fmm_dense_create)
  int n_blocks = 0;
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
  std::vector<int64_t> box_lin;   // [G] linear box index (ix * K + iy) * K + iz
  std::vector<double> theta, phi; // grid
  std::vector<double> dirs;       // [ndir][9]: k_hat, theta_hat, phi_hat
  // device copies for fmm_farfield_fill
  int device = -1;
  double* d_rowdata = nullptr;
  double* d_dirs = nullptr;
  double* d_waves = nullptr;      // plane waves of fmm_planewave_excitation, [cap][6]
  size_t waves_cap = 0;
};
