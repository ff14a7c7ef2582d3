// Mesh -> RWG basis functions -> FMM groups -> angular grid, and the far-field fill
// launcher (Section II.A and eq. (4)).  Host code; the arithmetic of eq. (4) runs in
// farfield_fill_kernel.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"
#include "kernels.hpp"

using namespace tuckfmm;

namespace {

// Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n, returned in decreasing
// order (so that theta = acos(x) increases).
std::vector<double> gauss_legendre_nodes(int n) {
  std::vector<double> x(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      // P_n'(z) = n (z P_n - P_{n-1}) / (z^2 - 1)
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  return x;
}

struct DirEdge {
  int64_t lo, hi;
  int32_t forward;  // 1 if the triangle traverses lo -> hi
  int32_t opp;
  int32_t tri;
};

}  // namespace

extern "C" fmm_status fmm_geometry_build(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                                         const double* origin, double box, int32_t boxes_per_axis,
                                         double wavenumber, int32_t n_theta, int32_t n_phi,
                                         fmm_geometry_t* out) {
  clear_error();
  if (!out) return fail(FMM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!verts || !tris || !origin) return fail(FMM_ERR_ARG, "verts, tris and origin must be non-NULL");
  if (n_verts < 3 || n_tris < 1) return fail(FMM_ERR_SHAPE, "need at least 3 vertices and 1 triangle");
  if (!(box > 0.0) || !std::isfinite(box)) return fail(FMM_ERR_ARG, "box must be positive and finite");
  if (boxes_per_axis < 1 || boxes_per_axis > 1 << 20) return fail(FMM_ERR_ARG, "boxes_per_axis out of range");
  if (!(wavenumber > 0.0) || !std::isfinite(wavenumber)) return fail(FMM_ERR_ARG, "wavenumber must be positive");
  if (n_theta < 1 || n_phi < 1 || (int64_t)n_theta * n_phi > (1 << 24))
    return fail(FMM_ERR_ARG, "angular grid size out of range");
  for (int64_t i = 0; i < 3 * n_verts; ++i)
    if (!std::isfinite(verts[i])) return fail(FMM_ERR_NUMERIC, "non-finite vertex coordinate");
  for (int64_t i = 0; i < 3 * n_tris; ++i)
    if (tris[i] < 0 || tris[i] >= n_verts) return fail(FMM_ERR_SHAPE, "triangle %lld references a bad vertex", (long long)(i / 3));

  auto* G = new fmm_geometry_s();
  G->n_verts = n_verts;
  G->n_tris = n_tris;
  G->verts.assign(verts, verts + 3 * n_verts);
  G->tris.assign(tris, tris + 3 * n_tris);
  std::memcpy(G->origin, origin, sizeof(G->origin));
  G->box = box;
  G->K = boxes_per_axis;
  G->k = wavenumber;
  G->n_theta = n_theta;
  G->n_phi = n_phi;

  // ---- RWG basis functions on the edges shared by two triangles
  std::vector<DirEdge> de(3 * n_tris);
  for (int64_t t = 0; t < n_tris; ++t) {
    const int32_t* v = tris + 3 * t;
    for (int e = 0; e < 3; ++e) {
      const int32_t u = v[e], w = v[(e + 1) % 3], o = v[(e + 2) % 3];
      DirEdge d;
      d.lo = std::min(u, w);
      d.hi = std::max(u, w);
      d.forward = u < w ? 1 : 0;
      d.opp = o;
      d.tri = (int32_t)t;
      de[3 * t + e] = d;
    }
  }
  std::sort(de.begin(), de.end(), [](const DirEdge& a, const DirEdge& b) {
    if (a.lo != b.lo) return a.lo < b.lo;
    if (a.hi != b.hi) return a.hi < b.hi;
    if (a.forward != b.forward) return a.forward > b.forward;
    return a.tri < b.tri;
  });
  // an edge of two oppositely traversing triangles carries a basis function; an edge
  // of one triangle is on the rim of an open surface and carries none
  std::vector<int64_t> elo, ehi;
  std::vector<int32_t> tp, tm, fp, fm;
  for (size_t i = 0; i < de.size();) {
    size_t j = i + 1;
    while (j < de.size() && de[j].lo == de[i].lo && de[j].hi == de[i].hi) ++j;
    if (de[i].lo == de[i].hi) {
      delete G;
      return fail(FMM_ERR_SHAPE, "degenerate triangle edge at vertex %d", de[i].lo);
    }
    if (j - i > 2) {
      delete G;
      return fail(FMM_ERR_SHAPE, "an edge is shared by more than two triangles");
    }
    if (j - i == 2) {
      const DirEdge& a = de[i];
      const DirEdge& b = de[i + 1];
      if (!(a.forward == 1 && b.forward == 0)) {
        delete G;
        return fail(FMM_ERR_SHAPE, "triangles are not consistently oriented");
      }
      elo.push_back(a.lo);
      ehi.push_back(a.hi);
      tp.push_back(a.tri);
      fp.push_back(a.opp);
      tm.push_back(b.tri);
      fm.push_back(b.opp);
    }
    i = j;
  }
  const int64_t ne = (int64_t)elo.size();
  if (ne == 0) {
    delete G;
    return fail(FMM_ERR_SHAPE, "the mesh has no edge shared by two triangles");
  }

  // ---- grouping by edge midpoint
  const int64_t K = boxes_per_axis;
  std::vector<int64_t> lin(ne);
  for (int64_t e = 0; e < ne; ++e) {
    int64_t idx[3];
    for (int c = 0; c < 3; ++c) {
      const double m = 0.5 * (G->verts[3 * elo[e] + c] + G->verts[3 * ehi[e] + c]);
      double f = std::floor((m - origin[c]) / box);
      int64_t i = (int64_t)f;
      if (f < 0.0) i = 0;
      if (f > (double)(K - 1)) i = K - 1;
      idx[c] = i;
    }
    lin[e] = (idx[0] * K + idx[1]) * K + idx[2];
  }
  std::vector<int64_t> perm(ne);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return lin[a] < lin[b]; });
  G->perm = perm;
  G->tri_p.resize(ne);
  G->tri_m.resize(ne);
  G->free_p.resize(ne);
  G->free_m.resize(ne);
  G->length.resize(ne);
  G->offsets.push_back(0);
  for (int64_t n = 0; n < ne; ++n) {
    const int64_t e = perm[n];
    G->tri_p[n] = tp[e];
    G->tri_m[n] = tm[e];
    G->free_p[n] = fp[e];
    G->free_m[n] = fm[e];
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double d = G->verts[3 * ehi[e] + c] - G->verts[3 * elo[e] + c];
      s += d * d;
    }
    G->length[n] = std::sqrt(s);
    if (n > 0 && lin[e] != lin[perm[n - 1]]) G->offsets.push_back(n);
    if (n == 0 || lin[e] != lin[perm[n - 1]]) {
      const int64_t L = lin[e];
      const int64_t ix = L / (K * K), iy = (L / K) % K, iz = L % K;
      G->centers.push_back(origin[0] + (ix + 0.5) * box);
      G->centers.push_back(origin[1] + (iy + 0.5) * box);
      G->centers.push_back(origin[2] + (iz + 0.5) * box);
      G->box_lin.push_back(L);
    }
  }
  G->offsets.push_back(ne);
  if (G->offsets.size() - 1 > (size_t)INT32_MAX) {
    delete G;
    return fail(FMM_ERR_SHAPE, "too many groups");
  }

  // ---- angular grid
  const std::vector<double> x = gauss_legendre_nodes(n_theta);
  G->theta.resize(n_theta);
  for (int i = 0; i < n_theta; ++i) G->theta[i] = std::acos(x[i]);
  G->phi.resize(n_phi);
  for (int j = 0; j < n_phi; ++j) G->phi[j] = 2.0 * M_PI * j / n_phi;
  G->dirs.resize((size_t)n_theta * n_phi * 9);
  for (int i = 0; i < n_theta; ++i)
    for (int j = 0; j < n_phi; ++j) {
      const double th = G->theta[i], ph = G->phi[j];
      const double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
      double* d = &G->dirs[((size_t)i * n_phi + j) * 9];
      d[0] = st * cp; d[1] = st * sp; d[2] = ct;
      d[3] = ct * cp; d[4] = ct * sp; d[5] = -st;
      d[6] = -sp;     d[7] = cp;      d[8] = 0.0;
    }
  *out = G;
  return FMM_OK;
}

extern "C" fmm_status fmm_geometry_info(fmm_geometry_t g, int64_t* n_basis, int32_t* n_groups) {
  clear_error();
  if (!g) return fail(FMM_ERR_ARG, "geometry is NULL");
  if (n_basis) *n_basis = g->offsets.back();
  if (n_groups) *n_groups = (int32_t)(g->offsets.size() - 1);
  return FMM_OK;
}

extern "C" fmm_status fmm_geometry_tables(fmm_geometry_t g, int64_t* offsets, int64_t* perm, double* centers,
                                          double* theta, double* phi) {
  clear_error();
  if (!g) return fail(FMM_ERR_ARG, "geometry is NULL");
  if (offsets) std::copy(g->offsets.begin(), g->offsets.end(), offsets);
  if (perm) std::copy(g->perm.begin(), g->perm.end(), perm);
  if (centers) std::copy(g->centers.begin(), g->centers.end(), centers);
  if (theta) std::copy(g->theta.begin(), g->theta.end(), theta);
  if (phi) std::copy(g->phi.begin(), g->phi.end(), phi);
  return FMM_OK;
}

extern "C" fmm_status fmm_geometry_boxes(fmm_geometry_t g, int32_t* boxes_per_axis, int64_t* box_of_group) {
  clear_error();
  if (!g) return fail(FMM_ERR_ARG, "geometry is NULL");
  if (boxes_per_axis) *boxes_per_axis = g->K;
  if (box_of_group) std::copy(g->box_lin.begin(), g->box_lin.end(), box_of_group);
  return FMM_OK;
}

extern "C" fmm_status fmm_geometry_layout(fmm_geometry_t g, fmm_layout* out) {
  clear_error();
  if (!g || !out) return fail(FMM_ERR_ARG, "geometry and out must be non-NULL");
  out->n_theta = g->n_theta;
  out->n_phi = g->n_phi;
  out->n_groups = (int32_t)(g->offsets.size() - 1);
  out->reserved = 0;
  out->offsets = g->offsets.data();
  return FMM_OK;
}

namespace {

// Per-row data of eq. (4) with the 3-point rule (see farfield_fill_kernel).
void row_data(const fmm_geometry_s* G, int64_t n, const double* c, double* out) {
  static const double B[3][3] = {{2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0},
                                 {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0},
                                 {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
  for (int side = 0; side < 2; ++side) {
    const int32_t tri = side == 0 ? G->tri_p[n] : G->tri_m[n];
    const int32_t fr = side == 0 ? G->free_p[n] : G->free_m[n];
    const double* corner[3];
    for (int k = 0; k < 3; ++k) corner[k] = &G->verts[3 * (int64_t)G->tris[3 * (int64_t)tri + k]];
    const double* p = &G->verts[3 * (int64_t)fr];
    for (int q = 0; q < 3; ++q) {
      double* e = out + (side * 3 + q) * 6;
      for (int x = 0; x < 3; ++x) {
        const double r = B[q][0] * corner[0][x] + B[q][1] * corner[1][x] + B[q][2] * corner[2][x];
        e[x] = r - c[x];
        e[3 + x] = side == 0 ? r - p[x] : p[x] - r;
      }
    }
  }
  out[36] = G->length[n] / 6.0;
  for (int x = 0; x < 3; ++x) out[37 + x] = c[x];  // the row's phase centre r_v
}

// Device copies of the per-row quadrature data and the direction table, built on the
// first device call (and again after a change of device).
fmm_status ensure_device_rows(fmm_geometry_s* g) {
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));
  if (g->d_rowdata != nullptr && g->device == dev) return FMM_OK;
  if (g->d_rowdata) {
    (void)hipFree(g->d_rowdata);
    (void)hipFree(g->d_dirs);
    g->d_rowdata = nullptr;
    g->d_dirs = nullptr;
  }
  if (g->d_waves) (void)hipFree(g->d_waves);
  g->d_waves = nullptr;
  g->waves_cap = 0;
  const int32_t ng = (int32_t)(g->offsets.size() - 1);
  const int64_t N = g->offsets.back();
  std::vector<double> rd((size_t)N * kRowDoubles);
  for (int32_t gr = 0; gr < ng; ++gr)
    for (int64_t n = g->offsets[gr]; n < g->offsets[gr + 1]; ++n)
      row_data(g, n, &g->centers[3 * (size_t)gr], &rd[(size_t)n * kRowDoubles]);
  TFMM_HIP(hipMalloc(&g->d_rowdata, rd.size() * sizeof(double)));
  TFMM_HIP(hipMalloc(&g->d_dirs, g->dirs.size() * sizeof(double)));
  TFMM_HIP(hipMemcpy(g->d_rowdata, rd.data(), rd.size() * sizeof(double), hipMemcpyHostToDevice));
  TFMM_HIP(hipMemcpy(g->d_dirs, g->dirs.data(), g->dirs.size() * sizeof(double), hipMemcpyHostToDevice));
  g->device = dev;
  return FMM_OK;
}

}  // namespace

extern "C" fmm_status fmm_farfield_fill(fmm_geometry_t g, int32_t first_group, int32_t count, void* farfield,
                                        void* stream) {
  clear_error();
  if (!g) return fail(FMM_ERR_ARG, "geometry is NULL");
  const int32_t ng = (int32_t)(g->offsets.size() - 1);
  if (first_group < 0 || count < 0 || (int64_t)first_group + count > ng)
    return fail(FMM_ERR_ARG, "group range [%d, %d) outside [0, %d)", first_group, first_group + count, ng);
  if (count == 0) return FMM_OK;
  if (!farfield) return fail(FMM_ERR_ARG, "farfield is NULL");
  if ((uintptr_t)farfield % 16) return fail(FMM_ERR_ARG, "farfield must be 16-byte aligned");
  if (!have_device()) return FMM_ERR_DEVICE;
  fmm_status st = ensure_device_rows(g);
  if (st != FMM_OK) return st;
  const int64_t row0 = g->offsets[first_group];
  const int64_t rows = g->offsets[first_group + count] - row0;
  TFMM_HIP(launch_farfield_fill(g->d_rowdata + row0 * kRowDoubles, rows, g->d_dirs, g->n_theta * g->n_phi, g->k,
                                farfield, static_cast<hipStream_t>(stream)));
  return FMM_OK;
}

extern "C" fmm_status fmm_planewave_excitation(fmm_geometry_t g, int32_t nrhs, const double* khat,
                                                const double* epol, fmm_prec prec, void* x, void* stream) {
  clear_error();
  if (!g) return fail(FMM_ERR_ARG, "geometry is NULL");
  if (nrhs < 1 || nrhs > 65535) return fail(FMM_ERR_ARG, "nrhs must be in [1, 65535]");
  if (!khat || !epol) return fail(FMM_ERR_ARG, "khat and epol must be non-NULL");
  if (prec < FMM_C128 || prec > FMM_BF16X3) return fail(FMM_ERR_ARG, "bad precision %d", (int)prec);
  const size_t es = prec == FMM_C128 ? 16 : 8;
  if (!x) return fail(FMM_ERR_ARG, "x is NULL");
  if ((uintptr_t)x % es) return fail(FMM_ERR_ARG, "x must be %zu-byte aligned", es);
  std::vector<double> waves((size_t)nrhs * 6);
  for (int32_t r = 0; r < nrhs; ++r) {
    double kk = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double kv = khat[3 * (size_t)r + c], ev = epol[3 * (size_t)r + c];
      if (!std::isfinite(kv) || !std::isfinite(ev))
        return fail(FMM_ERR_NUMERIC, "non-finite direction or polarisation of wave %d", r);
      kk += kv * kv;
      waves[6 * (size_t)r + c] = kv;
      waves[6 * (size_t)r + 3 + c] = ev;
    }
    if (std::fabs(std::sqrt(kk) - 1.0) > 1e-6) return fail(FMM_ERR_ARG, "direction of wave %d is not a unit vector", r);
  }
  if (!have_device()) return FMM_ERR_DEVICE;
  fmm_status st = ensure_device_rows(g);
  if (st != FMM_OK) return st;
  if ((size_t)nrhs > g->waves_cap) {
    if (g->d_waves) (void)hipFree(g->d_waves);
    g->d_waves = nullptr;
    g->waves_cap = 0;
    TFMM_HIP(hipMalloc(&g->d_waves, waves.size() * sizeof(double)));
    g->waves_cap = (size_t)nrhs;
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  // the table is copied before the kernel may read it (a stream-ordered copy from
  // pageable memory returns once the source has been consumed)
  TFMM_HIP(hipStreamSynchronize(hs));
  TFMM_HIP(hipMemcpy(g->d_waves, waves.data(), waves.size() * sizeof(double), hipMemcpyHostToDevice));
  TFMM_HIP(launch_planewave(g->d_rowdata, g->offsets.back(), g->d_waves, nrhs, g->k, es, x, hs));
  return FMM_OK;
}

extern "C" void fmm_geometry_destroy(fmm_geometry_t g) {
  if (!g) return;
  if (g->d_rowdata) (void)hipFree(g->d_rowdata);
  if (g->d_dirs) (void)hipFree(g->d_dirs);
  if (g->d_waves) (void)hipFree(g->d_waves);
  delete g;
}
